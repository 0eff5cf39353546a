// HIP kernels of the multirate MRT lattice-Boltzmann hot path (gfx950).
//
// Every kernel processes one 64 x TY tile per block (256 threads = four
// wavefronts, one wavefront per row across x), so every global access to a
// plane is a coalesced 256-byte (FP32) row segment.  The stencil kernels
// stage the tile plus its halo in LDS: macroscopic planes two rings deep for
// the isotropic gradient, and post-collision values one ring deep so that the
// pull streaming reads its neighbours from LDS.  Halo collisions are
// recomputed (about 2 (TX + TY) / (TX TY) extra work) instead of being written
// to and re-read from HBM.
//
// State representation (see lbm_dev.h):
//   phase:  phi in a compute-precision plane, plus s_i = f_i - w_i phi for
//           i = 1..4 in the storage type (the rest population is
//           w_0 phi - sum s_i, so sum_i f_i = phi exactly);
//   U, T:   the zeroth moment chi in a compute-precision plane and the first
//           moment j in the storage type.  With the relaxation of Eq. (23)
//           only these moments enter the collision, so the post-collision
//           populations are w_i (chi + dt Q) + e_i . [j_eq + (1 - s)(j - j_eq)] / 2
//           (D2Q5) and the state after streaming is again (chi, j);
//   flow:   rho plus s_i = f_i - w_i rho for i = 1..8 (D2Q9), and u.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <type_traits>

#include "lbm_dev.h"

namespace lbm {

// ------------------------------------------------------------------ storage
// Every plane is device global memory.  The plane pointers live in the
// domain descriptor, so the compiler sees generic pointers and would emit
// flat loads and stores (which also wait on the LDS counter); gp() casts
// them to the global address space so they become global_load/store.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T* gp(const void* p) {
  return (GLOBAL T*)(T*)p;
}

__device__ __forceinline__ double ld(const GLOBAL double* p, long long i) { return p[i]; }
__device__ __forceinline__ float ld(const GLOBAL float* p, long long i) { return p[i]; }
// (the 16-bit formats move as raw bits: their class types have no
// address-space-qualified copy constructors)
__device__ __forceinline__ float ld(const GLOBAL __half* p, long long i) {
  return __half2float(__ushort_as_half(((const GLOBAL uint16_t*)p)[i]));
}
__device__ __forceinline__ float ld(const GLOBAL __hip_bfloat16* p, long long i) {
  return __uint_as_float((uint32_t)((const GLOBAL uint16_t*)p)[i] << 16);
}
__device__ __forceinline__ void st(GLOBAL double* p, long long i, double v) { p[i] = v; }
__device__ __forceinline__ void st(GLOBAL float* p, long long i, float v) { p[i] = v; }
__device__ __forceinline__ void st(GLOBAL __half* p, long long i, float v) {
  ((GLOBAL uint16_t*)p)[i] = __half_as_ushort(__float2half(v));
}
__device__ __forceinline__ double ld(const double* p, long long i) { return p[i]; }
__device__ __forceinline__ float ld(const float* p, long long i) { return p[i]; }
__device__ __forceinline__ float ld(const __half* p, long long i) { return __half2float(p[i]); }
__device__ __forceinline__ float ld(const __hip_bfloat16* p, long long i) { return __bfloat162float(p[i]); }

__device__ __forceinline__ void st(double* p, long long i, double v) { p[i] = v; }
__device__ __forceinline__ void st(float* p, long long i, float v) { p[i] = v; }
__device__ __forceinline__ void st(__half* p, long long i, float v) { p[i] = __float2half(v); }
// BF16 stores round stochastically.  Round-to-nearest gives every stored
// value the same error for as long as the field is quasi-steady, and those
// repeated errors in the scalar fluxes add up to a steady drift of the total
// solute; with the rounding direction drawn with probability proportional to
// the distance to each neighbour the error has zero mean and does not
// repeat.  The 16 random bits hash the FP32 value with its element index
// (Wellons' lowbias32 integer hash), so a store is a pure function of what
// is stored and where: runs stay bitwise reproducible across tile shapes.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// gfx950's v_cvt_sr_bf16_f32 adds the top 16 bits of r below the kept
// mantissa of a finite value and truncates (infinities and NaN pass
// through): the integer form of this rounding in one instruction, bit for
// bit.
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2_t;
__device__ __forceinline__ uint16_t bf16_sr_hw(float v, uint32_t r) {
  const bf16x2_t b = __builtin_amdgcn_cvt_sr_bf16_f32((bf16x2_t){0, 0}, v, r, false);
  return (uint16_t)(__builtin_bit_cast(uint32_t, b) & 0xffffu);
}
__device__ __forceinline__ uint16_t bf16_sr(float v, long long i) {
  const uint32_t u = __float_as_uint(v);
  return bf16_sr_hw(v, mix32(u + 0x9e3779b9u * (uint32_t)i) << 16);
}
__device__ __forceinline__ void st(__hip_bfloat16* p, long long i, float v) { ((uint16_t*)p)[i] = bf16_sr(v, i); }
__device__ __forceinline__ void st(GLOBAL __hip_bfloat16* p, long long i, float v) {
  ((GLOBAL uint16_t*)p)[i] = bf16_sr(v, i);
}

// Stochastic BF16 rounding of the 3D kernels: one stream of random words
// per site and launch.  The stream starts at a hash of the site's offset,
// the absolute base step and a per-kernel constant, and advances by the
// golden-ratio increment per store (a Weyl sequence: one add); gfx950's
// v_cvt_sr_bf16_f32 adds the word's top 16 bits below the kept mantissa
// and truncates (the rounding of bf16_sr, in one instruction).  Each word
// is uniform over steps since its start is, so every store rounds up with
// the probability of its remainder (unbiased), while the words of one site
// are spread evenly.  A store is a pure function of the site, the step and
// the value, so runs stay bitwise reproducible across launch shapes and
// graph replays, and a value held constant over many steps is still
// rounded up and down in proportion.  One hash per site instead of one per
// store: the D3Q19 flow stores 18 values per site.
struct SRStream {
  uint32_t s;
  __device__ __forceinline__ uint32_t next() {
    s += 0x9e3779b9u;
    return s;
  }
};
__device__ __forceinline__ SRStream sr_stream(unsigned o, long long step, uint32_t salt) {
  return SRStream{mix32(o ^ ((uint32_t)step * 0x9e3779b9u) ^ salt)};
}

// Element i of a plane addressed through a 32-bit byte offset.  The plane
// base is uniform and stays in scalar registers, and one vector register
// holding the offset serves every plane of a site, so each access is one
// global load or store in base + offset form with no 64-bit address
// arithmetic per lane.  Every 2D plane is smaller than 4 GiB (lbm_create
// rejects larger ones).
template <class T>
__device__ __forceinline__ const GLOBAL T* at(const GLOBAL T* p, unsigned i) {
  return (const GLOBAL T*)((const GLOBAL char*)p + i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ GLOBAL T* at(GLOBAL T* p, unsigned i) {
  return (GLOBAL T*)((GLOBAL char*)p + i * (unsigned)sizeof(T));
}
// The plane at element offset off of a group of planes.  The optimiser
// would otherwise fold the per-lane offset of a site into one 64-bit vector
// address and add each plane's stride to it per lane; the empty asm
// statement (it emits no instruction) keeps every plane base a separate
// scalar value, so all the planes of a site share the one offset register.
template <class T>
__device__ __forceinline__ T* plane(T* p, long long off) {
  T* r = p + off;
  asm("" : "+s"(r));
  return r;
}
__device__ __forceinline__ double ldo(const GLOBAL double* p, unsigned i) { return *at(p, i); }
__device__ __forceinline__ float ldo(const GLOBAL float* p, unsigned i) { return *at(p, i); }
__device__ __forceinline__ float ldo(const GLOBAL __half* p, unsigned i) {
  return __half2float(__ushort_as_half(*at((const GLOBAL uint16_t*)p, i)));
}
__device__ __forceinline__ float ldo(const GLOBAL __hip_bfloat16* p, unsigned i) {
  return __uint_as_float((uint32_t)*at((const GLOBAL uint16_t*)p, i) << 16);
}
__device__ __forceinline__ void sto(GLOBAL double* p, unsigned i, double v) { *at(p, i) = v; }
__device__ __forceinline__ void sto(GLOBAL float* p, unsigned i, float v) { *at(p, i) = v; }
__device__ __forceinline__ void sto(GLOBAL __half* p, unsigned i, float v) {
  *at((GLOBAL uint16_t*)p, i) = __half_as_ushort(__float2half(v));
}
__device__ __forceinline__ void sto(GLOBAL __hip_bfloat16* p, unsigned i, float v) {
  *at((GLOBAL uint16_t*)p, i) = bf16_sr(v, i);
}

// Stores that draw their rounding from a site's stream (3D kernels): BF16
// rounds stochastically with the next word, every other format as sto().
template <class T, class V>
__device__ __forceinline__ void sto_sr(GLOBAL T* p, unsigned i, V v, SRStream&) {
  sto(p, i, v);
}
__device__ __forceinline__ void sto_sr(GLOBAL __hip_bfloat16* p, unsigned i, float v, SRStream& rs) {
  *at((GLOBAL uint16_t*)p, i) = bf16_sr_hw(v, rs.next());
}

// Raw storage bits of a population plane (16-bit formats as their bit
// patterns), so that prefetched loads are not consumed by a conversion
// before they are needed; cvt_raw converts at the point of use.
template <class S> struct RawT { using type = S; };
template <> struct RawT<__half> { using type = uint16_t; };
template <> struct RawT<__hip_bfloat16> { using type = uint16_t; };
__device__ __forceinline__ double cvt_raw(double v, double*) { return v; }
__device__ __forceinline__ float cvt_raw(float v, float*) { return v; }
__device__ __forceinline__ float cvt_raw(uint16_t v, __half*) { return __half2float(__ushort_as_half(v)); }
__device__ __forceinline__ float cvt_raw(uint16_t v, __hip_bfloat16*) { return __uint_as_float((uint32_t)v << 16); }

// Reciprocal and inverse square root: the hardware approximations (about
// 1 ulp) in the FP32 path, exact division and square root in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Ghost index for stencils: wrap on periodic axes, clamp (even mirror about
// the half-way wall) otherwise.  Callers stay within two nodes of the domain
// and every side is at least three nodes long.
__device__ __forceinline__ int ghost(int g, int n, int bc) {
  if (g < 0) return bc == BC_PER ? g + n : 0;
  if (g >= n) return bc == BC_PER ? g - n : n - 1;
  return g;
}

// Site a raw coordinate refers to: wrapped on periodic axes, -1 beyond a wall.
__device__ __forceinline__ int resolve(int g, int n, int bc) {
  if (g < 0) return bc == BC_PER ? g + n : -1;
  if (g >= n) return bc == BC_PER ? g - n : -1;
  return g;
}

template <class R>
__device__ __forceinline__ void iso_grad(const R* b, int stride, R& gx, R& gy) {
  // isotropic gradient with D2Q9 weights, b points at the centre
  const R E = b[1], W = b[-1], N = b[stride], S = b[-stride];
  const R NE = b[stride + 1], NW = b[stride - 1], SE = b[-stride + 1], SW = b[-stride - 1];
  gx = (E - W) * R(1.0 / 3.0) + (NE - NW - SW + SE) * R(1.0 / 12.0);
  gy = (N - S) * R(1.0 / 3.0) + (NE + NW - SW - SE) * R(1.0 / 12.0);
}

// e . (a, b) and e . (a, b, c) for a lattice direction e.  The components
// are compile-time constants once the direction loops are unrolled, so the
// zero ones are dropped here: the compiler keeps a multiply by zero (0 * x
// is not 0 for every x in IEEE arithmetic) and with it the load of x.  The
// result equals the full sum for every finite input.
template <class R>
__device__ __forceinline__ R edot2(int ex, int ey, R a, R b) {
  if (ex == 0) return ey == 0 ? R(0) : R(ey) * b;
  if (ey == 0) return R(ex) * a;
  return R(ex) * a + R(ey) * b;
}
template <class R>
__device__ __forceinline__ R edot3(int ex, int ey, int ez, R a, R b, R c) {
  if (ex == 0) return edot2(ey, ez, b, c);
  if (ey == 0 && ez == 0) return R(ex) * a;
  if (ey == 0) return R(ex) * a + R(ez) * c;
  if (ez == 0) return R(ex) * a + R(ey) * b;
  return R(ex) * a + R(ey) * b + R(ez) * c;
}

// D2Q5: e_1 = +x, e_2 = +y, e_3 = -x, e_4 = -y (compile-time tables so that
// unrolled loops fold them into immediates).
#define EX5(q) ((q) == 1 ? 1 : (q) == 3 ? -1 : 0)
#define EY5(q) ((q) == 2 ? 1 : (q) == 4 ? -1 : 0)
// D2Q9 (Eq. 15): 0, the axes as in D2Q5, then (1,1), (-1,1), (-1,-1), (1,-1)
#define EX9(q) ((q) == 1 || (q) == 5 || (q) == 8 ? 1 : (q) == 3 || (q) == 6 || (q) == 7 ? -1 : 0)
#define EY9(q) ((q) == 2 || (q) == 5 || (q) == 6 ? 1 : (q) == 4 || (q) == 7 || (q) == 8 ? -1 : 0)

// Scalar lattices of the phase, U and T fields: D2Q5 (weights 1/3, 1/6) or
// the paper's D2Q9 (4/9, 1/9, 1/36).  With the relaxation of Eq. (23) every
// moment but the flux relaxes to equilibrium, so the post-collision
// populations depend on (chi, j) only:
//   f_i^+ = w_i (chi + dP) + e_i . [ (3 w_i - c_K) j_eq + c_K K ],
//   K = j_eq + (1 - 1/tau)(j - j_eq),
// where c_K = 1 / sum_k e_kx^2 is 1/2 (D2Q5) or 1/6 (D2Q9) (the flux row of
// the moment basis has that squared norm); in D2Q5 3 w_i = c_K, so only K
// enters.
template <int Q>
struct Lat2 {
  static constexpr int ex(int q) { return Q == 5 ? EX5(q) : EX9(q); }
  static constexpr int ey(int q) { return Q == 5 ? EY5(q) : EY9(q); }
  static constexpr double w(int q) {
    return Q == 5 ? (q == 0 ? 1.0 / 3 : 1.0 / 6) : (q == 0 ? 4.0 / 9 : q <= 4 ? 1.0 / 9 : 1.0 / 36);
  }
  static constexpr double cK = Q == 5 ? 0.5 : 1.0 / 6;
  static constexpr double cJ(int q) { return 3.0 * w(q) - cK; }   // 0 in D2Q5
};

// =================================================================== phase
// Collision of Eq. (14) with the equilibrium of Eq. (21), the relaxation of
// Eq. (23), tau_phi of Eq. (24) and the source dt w_i Q_phi / tau0, then the
// anisotropic streaming of Eq. (26) in pull form with a_s^2 at the
// destination.  The result per site of the collision is (dP, K):
// f_i^+ = w_i (phi + dP) + e_i . K / 2 with dP = dt Q / tau0 and
// K = j_eq + (1 - 1/tau)(j - j_eq), j_eq = v_n dt.
//
// Deviation form: every population is handled as its deviation from
// w_i times the zeroth moment of the site it is written to, and the new
// zeroth moment is the old one plus the sum of the deviations.  This is
// the same arithmetic rearranged; a uniform state is then reproduced
// exactly in any precision instead of drifting by the rounding of
// w_i chi summed over i at every step.
template <class R>
struct PhaseConst {
  R dt, W2t, inv_tau0, eps, lam, Mc, cth, sth, inv_lhcp, theta_off, Wt;
};

template <class R>
__device__ __forceinline__ PhaseConst<R> phase_const(const Dom& D) {
  PhaseConst<R> c;
  c.dt = kc<R>(D, K_DTPHI);
  c.W2t = kc<R>(D, K_W2T);
  c.inv_tau0 = kc<R>(D, K_INVTAU0);
  c.eps = kc<R>(D, K_EPS);
  c.lam = kc<R>(D, K_LAM);
  c.Mc = kc<R>(D, K_MC);
  c.cth = kc<R>(D, K_CTH);
  c.sth = kc<R>(D, K_STH);
  c.inv_lhcp = kc<R>(D, K_INVLHCP);
  c.theta_off = kc<R>(D, K_THOFF);
  return c;
}

template <class R>
__device__ __forceinline__ void phase_collide(const PhaseConst<R>& c, R phi, R gx, R gy, R jx, R jy,
                                              R Us, R Ts, R& dP, R& Kx, R& Ky, R& A, R* jeq = nullptr) {
  const R gg = gx * gx + gy * gy;
  R a_s = R(1), Nx = R(0), Ny = R(0);
  if (gg >= R(GRAD_EPS2)) {
    const R ig = rsq(gg);
    const R g = gg * ig;
    const R nx = -gx * ig, ny = -gy * ig;
    const R ax = c.cth * nx + c.sth * ny;
    const R ay = -c.sth * nx + c.cth * ny;
    const R ax2 = ax * ax, ay2 = ay * ay;
    const R s4 = ax2 * ax2 + ay2 * ay2;
    a_s = R(1) - R(3) * c.eps + R(4) * c.eps * s4;
    const R f = R(-16) * c.eps * a_s * g;
    const R nxc = f * ax * (ax2 - s4);
    const R nyc = f * ay * (ay2 - s4);
    Nx = c.cth * nxc - c.sth * nyc;
    Ny = c.sth * nxc + c.cth * nyc;
  }
  A = a_s * a_s;
  const R tau = R(3) * c.dt * A * c.W2t + R(0.5);
  const R om = R(1) - rcp(tau);
  // v_n = -W0^2 N / tau0 ; j_eq = v_n dt
  const R jex = -c.W2t * Nx * c.dt;
  const R jey = -c.W2t * Ny * c.dt;
  const R theta = (Ts - c.theta_off) * c.inv_lhcp;
  const R q = R(1) - phi * phi;
  const R Q = phi * q - c.lam * (c.Mc * Us + theta) * q * q;
  dP = c.dt * Q * c.inv_tau0;
  Kx = jex + om * (jx - jex);
  Ky = jey + om * (jy - jey);
  if (jeq) {
    jeq[0] = jex;
    jeq[1] = jey;
  }
}

// Ring cell r of the collision box of a w x h tile (box cells (lx, ly) in
// [0, w+1] x [0, h+1], the tile being 1..w x 1..h): top row, bottom row,
// left column, right column.  There are 2 (w + 2) + 2 h <= 196 of them, so
// every thread of a block handles at most one.
__device__ __forceinline__ bool ring_cell(int r, int w, int h, int& lx, int& ly) {
  const int W2 = w + 2;
  if (r < W2) { lx = r; ly = 0; return true; }
  r -= W2;
  if (r < W2) { lx = r; ly = h + 1; return true; }
  r -= W2;
  if (r < h) { lx = 0; ly = 1 + r; return true; }
  r -= h;
  if (r < h) { lx = w + 1; ly = 1 + r; return true; }
  return false;
}

// Load the tile's field plane plus two rings (ghosts wrapped or mirrored)
// into LDS, BW = TX + 4 columns (thread column tx and, for tx < 4, tx + 64)
// by BH rows.  Issued before the first barrier together with every other
// global load of the block, so a block waits for memory once.
template <class R, int BW, int BH>
__device__ __forceinline__ void load_box2(R* box, const GLOBAL R* __restrict__ src, int px, int x0, int y0, int nx,
                                          int ny, int bcx, int bcy, int tx, int ty) {
  static_assert(BW == TX + 4, "box width");
  const int gx0 = ghost(x0 - 2 + tx, nx, bcx);
  const bool two = tx < BW - TX;
  const int gx1 = two ? ghost(x0 - 2 + tx + TX, nx, bcx) : 0;
#pragma unroll
  for (int r = 0; r < (BH + BY - 1) / BY; ++r) {   // rows ty, ty + BY, ... below BH
    const int ly = ty + r * BY;
    if (ly >= BH) break;
    const unsigned row = (unsigned)(ghost(y0 - 2 + ly, ny, bcy) * px);
    box[ly * BW + tx] = ldo(src, row + gx0);
    if (two) box[ly * BW + tx + TX] = ldo(src, row + gx1);
  }
}

// =================================================================== phase kernel
template <class R, class S, int TY, int Q>
__global__ __launch_bounds__(NTHR) void k_phase(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                 unsigned k) {
  using Lq = Lat2<Q>;
  constexpr int RPT = TY / BY;
  constexpr int NS = RPT + 1;  // owned sites + one ring cell per thread
  constexpr int BW = TX + 4, BH = TY + 4;
  constexpr int CW = TX + 2, CH = TY + 2;
  constexpr int NJ = Q == 9 ? CH * CW : 1;
  __shared__ R sphi[BH * BW];
  __shared__ R sP[CH * CW], sKx[CH * CW], sKy[CH * CW];
  __shared__ R sJx[NJ], sJy[NJ];   // D2Q9: j_eq of the collision

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  if (k % D.N_phi) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px, pl = (int)D.plane;
  const int x0 = t.y, y0 = t.z;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int bcx = D.bc[0], bcy = D.bc[1];
  const unsigned np = n_phi(D, k - 1);
  const int ib = par(np), ob = ib ^ 1;
  GLOBAL const R* __restrict__ phi_in = gp<const R>(D.phi[qb(np)]);
  GLOBAL R* __restrict__ phi_out = gp<R>(D.phi[qb(np + 1)]);
  GLOBAL const S* __restrict__ s_in = gp<const S>(D.sphi[ib]);
  GLOBAL S* __restrict__ s_out = gp<S>(D.sphi[ob]);
  // latest U and T (before this step's transfer)
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  GLOBAL const R* __restrict__ Up = D.has_U ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL const R* __restrict__ Tp = D.has_T ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;

  const PhaseConst<R> c = phase_const<R>(D);
  // variant: grad phi from Eq. (40) with the previous phase step's v_n dt
  // and A at the site (written by that step into the other buffer)
  const bool e40 = D.gradeq40 != 0;
  GLOBAL const R* __restrict__ gq_in = e40 ? gp<const R>(D.gq[ib]) : nullptr;
  GLOBAL R* __restrict__ gq_out = e40 ? gp<R>(D.gq[ob]) : nullptr;

  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  // sites of this thread: RPT owned sites, then at most one ring cell
  int cl[NS];                 // collision-box index (-1: inactive)
  int bi[NS];                 // the same cell in the phi box
  unsigned so[NS];            // in-plane offset
  R sv[NS][Q - 1], Uv[NS], Tv[NS], gqv[NS][3];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    int lx, ly, gx, gy;
    cl[r] = -1;
    if (r < RPT) {
      lx = tx + 1;
      ly = ty + r * BY + 1;
      if (tx >= w || ly > h) continue;
      gx = x0 + tx;
      gy = y0 + ly - 1;
    } else {
      if (!ring_cell(tid, w, h, lx, ly)) continue;
      gx = resolve(x0 - 1 + lx, nx, bcx);
      gy = resolve(y0 - 1 + ly, ny, bcy);
      if (gx < 0 || gy < 0) continue;  // beyond a wall: never pulled from
    }
    cl[r] = ly * CW + lx;
    bi[r] = (ly + 1) * BW + lx + 1;
    const unsigned o = gy * px + gx;
    so[r] = o;
#pragma unroll
    for (int q = 0; q < Q - 1; ++q) sv[r][q] = ldo(plane(s_in, q * pl), o);
    Uv[r] = Up ? ldo(Up, o) + kc<R>(D, K_U0) : R(0);      // planes hold U - U0 and T - T0
    Tv[r] = Tp ? ldo(Tp, o) + kc<R>(D, K_T0) : c.theta_off;
    if (e40) {
#pragma unroll
      for (int a = 0; a < 3; ++a) gqv[r][a] = ldo(plane(gq_in, a * pl), o);
    }
  }
  load_box2<R, BW, BH>(sphi, phi_in, px, x0, y0, nx, ny, bcx, bcy, tx, ty);
  __syncthreads();

  R Aown[RPT];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (cl[r] < 0) continue;
    const R* b = &sphi[bi[r]];
    R jx, jy;   // first moment of the deviations (the w_i phi part has none)
    if constexpr (Q == 5) {
      jx = sv[r][0] - sv[r][2];
      jy = sv[r][1] - sv[r][3];
    } else {
      jx = sv[r][0] - sv[r][2] + sv[r][4] - sv[r][5] - sv[r][6] + sv[r][7];
      jy = sv[r][1] - sv[r][3] + sv[r][4] + sv[r][5] - sv[r][6] - sv[r][7];
    }
    R gx_, gy_;
    if (e40) {   // Eq. (40): grad phi = -(3 / tau_prev) (j - v_n,prev dt)
      const R f = R(-3) / (R(3) * c.dt * gqv[r][2] * c.W2t + R(0.5));
      gx_ = f * (jx - gqv[r][0]);
      gy_ = f * (jy - gqv[r][1]);
    } else {
      iso_grad(b, BW, gx_, gy_);
    }
    R dP, Kx, Ky, A, je[2];
    phase_collide(c, b[0], gx_, gy_, jx, jy, Uv[r], Tv[r], dP, Kx, Ky, A, je);
    if (e40 && r < RPT) {
      sto(gq_out, so[r], je[0]);
      sto(plane(gq_out, pl), so[r], je[1]);
      sto(plane(gq_out, 2 * pl), so[r], A);
    }
    sP[cl[r]] = dP;
    sKx[cl[r]] = Kx;
    sKy[cl[r]] = Ky;
    if constexpr (Q == 9) {
      sJx[cl[r]] = je[0];
      sJy[cl[r]] = je[1];
    }
    if (r < RPT) Aown[r] = A;
  }
  __syncthreads();

  // anisotropic pull streaming (Eq. 26) into owned sites, in deviations
  // d_i = f_i - w_i phi(y) of the destination y:
  //   A d_i^new = [f_i^+(y - e_i) - w_i phi(y)] - (1 - A) d_i
  // Only tiles on a wall test the upstream node of each direction (a test
  // uniform over the block).
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;
  const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y0 == 0 || y0 + h >= ny));
  auto stream = [&](auto edge_c) {
    constexpr bool EDGE = decltype(edge_c)::value;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (cl[r] < 0) continue;
      const int ci = cl[r];
      const int bc = bi[r];
      const int gx = x0 + tx, gy = y0 + ty + r * BY;
      const R A = Aown[r], iA = rcp(A), oA = R(1) - A;
      const R phy = sphi[bc];
      const R dPo = sP[ci];
      R s0 = R(0);
#pragma unroll
      for (int q = 0; q < Q - 1; ++q) s0 -= sv[r][q];
      R dn[Q];
      dn[0] = (dPo * R(Lq::w(0)) - oA * s0) * iA;
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        const int ex = Lq::ex(q), ey = Lq::ey(q);
        // upstream node gx - ex, gy - ey beyond a wall: half-way bounce-back
        // from this node
        const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                   (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
        R dpost;
        if (wall) {
          dpost = dPo * R(Lq::w(q)) - R(Lq::cK) * edot2(ex, ey, sKx[ci], sKy[ci]);
          if constexpr (Q == 9) dpost -= R(Lq::cJ(q)) * edot2(ex, ey, sJx[ci], sJy[ci]);
        } else {
          const int si = ci - ey * CW - ex;
          const R dphi = sphi[bc - ey * BW - ex] - phy;
          dpost = (dphi + sP[si]) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, sKx[si], sKy[si]);
          if constexpr (Q == 9) dpost += R(Lq::cJ(q)) * edot2(ex, ey, sJx[si], sJy[si]);
        }
        dn[q] = (dpost - oA * sv[r][q - 1]) * iA;
      }
      R dphin = dn[0];
#pragma unroll
      for (int q = 1; q < Q; ++q) dphin += dn[q];
      const unsigned o = gy * px + gx;
      sto(phi_out, o, phy + dphin);
#pragma unroll
      for (int q = 1; q < Q; ++q) sto(plane(s_out, (q - 1) * pl), o, dn[q] - dphin * R(Lq::w(q)));
    }
  };
  if (edge) stream(std::true_type{});
  else stream(std::false_type{});
}

// =================================================================== 2D marching in y
// For large domains: one block owns a column of YOW = 62 sites over a run
// of rows (the host lists the runs) and walks up through it four rows at a
// time (one row per wavefront).  The phase field is kept in an eight-row
// LDS ring (the column plus two cells on each side), the collisions of the
// four rows ahead go into an eight-row LDS ring (the column plus one ring
// cell on each side: 64 cells, one per lane), and the four current rows are
// streamed from the rows below, at and above.  Ring collisions are
// recomputed only in x (3% instead of 16% for a 64 x 16 tile), and the
// loads of the next four rows are issued before the current rows are
// computed.  The arithmetic is the tile kernels', expression for
// expression.
// A run is YOW = 62 columns wide, so that its collision row (the columns
// plus one ring cell on each side) is exactly one wavefront of 64 lanes:
// lane tx holds collision column tx, lanes 1 .. w the own columns.  (With
// 64-column runs the two ring cells of every row cost wave 0 a second
// collision pass, a quarter more collision work per block.)
constexpr int YOW = TX - 2, YCW = TX, YBW = TX + 2;
static_assert(YOW == YCOL, "run width shared with the host");

// Slot of a run's largest |dU| (and injected U) in the per-run maxima that
// the diagnostics reduce: the domain's runs are numbered row by row.
__device__ __forceinline__ int ym_run(const Dom& D, int x0, int ya) {
  return D.rbase + (ya / YRUN) * ((D.nx + YOW - 1) / YOW) + x0 / YOW;
}

// isotropic gradient with D2Q9 weights from three rows (below, at, above)
template <class R>
__device__ __forceinline__ void iso_grad_rows(const R* rm, const R* r0, const R* rp, int c, R& gx, R& gy) {
  const R E = r0[c + 1], W = r0[c - 1], N = rp[c], S = rm[c];
  const R NE = rp[c + 1], NW = rp[c - 1], SE = rm[c + 1], SW = rm[c - 1];
  gx = (E - W) * R(1.0 / 3.0) + (NE - NW - SW + SE) * R(1.0 / 12.0);
  gy = (N - S) * R(1.0 / 3.0) + (NE + NW - SW - SE) * R(1.0 / 12.0);
}

// collision cell of a thread for the four rows r0 .. r0 + 3: column tx of
// row r0 + ty (columns 0 and w + 1 are the ring cells of a run w wide).
// There is one cell per thread; the second slot (i = 1) of the callers'
// loops is never taken.
__device__ __forceinline__ bool ym_cell(int i, int tx, int ty, int tid, int w, int r0, int& col, int& row) {
  col = tx;
  row = r0 + ty;
  return i == 0 && tx <= w + 1;
}

// The marching phase kernel keeps runs 64 columns wide: its own columns
// start on 64-element boundaries, so its five output planes are written in
// whole lines (with 62-column runs it moved 11-19% more bytes in writes).
// The two ring cells of each of its rows take a second pass of wave 0.
constexpr int PCW = TX + 2, PBW = TX + 4;
__device__ __forceinline__ bool ym_cell64(int i, int tx, int ty, int tid, int w, int r0, int& col, int& row) {
  if (i == 0) {
    col = tx + 1;
    row = r0 + ty;
    return tx < w;
  }
  if (tid >= 8) return false;
  col = (tid & 1) ? w + 1 : 0;
  row = r0 + (tid >> 1);
  return true;
}

template <class R, class S, int Q>
struct YPhaseIn {
  typename RawT<S>::type s[2][Q - 1];
  R U[2], T[2];
  R phi[2];   // two phase-field window cells
};

template <class R, class S, int Q>
__device__ __forceinline__ void ym_load_phase(int nx, int ny, int px, int bcx, int bcy, int x0, int w, int r0,
                                              long long pl, int tx, int ty, int tid,
                                              GLOBAL const R* phi, GLOBAL const typename RawT<S>::type* sp,
                                              GLOBAL const R* Up, GLOBAL const R* Tp, YPhaseIn<R, S, Q>& in,
                                              bool inputs = true) {
  // collision inputs of rows r0 .. r0 + 3
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!inputs) break;
    int col, row;
    if (!ym_cell64(i, tx, ty, tid, w, r0, col, row)) continue;
    const int gx = resolve(x0 - 1 + col, nx, bcx), gy = resolve(row, ny, bcy);
    if (gx < 0 || gy < 0) continue;
    const unsigned o = (unsigned)gy * (unsigned)px + (unsigned)gx;
#pragma unroll
    for (int q = 0; q < Q - 1; ++q) in.s[i][q] = *at(plane(sp, q * pl), o);
    if (Up) in.U[i] = ldo(Up, o);
    if (Tp) in.T[i] = ldo(Tp, o);
  }
  // phase-field rows r0 + 1 .. r0 + 4 (68 cells each, ghosted)
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int cc = tid + 256 * i;
    if (cc < 4 * PBW) {
      const int gx = ghost(x0 - 2 + cc % PBW, nx, bcx), gy = ghost(r0 + 1 + cc / PBW, ny, bcy);
      in.phi[i] = ldo(phi, (unsigned)gy * (unsigned)px + (unsigned)gx);
    }
  }
}

template <class R, class S, int Q>
__device__ __forceinline__ void k_phase_ym_run(const Dom* __restrict__ doms, const int4 t, unsigned k) {
  using Lq = Lat2<Q>;
  using SR = typename RawT<S>::type;
  constexpr int NV = Q == 9 ? 5 : 3;   // dP, Kx, Ky (and j_eq in D2Q9)
  __shared__ R wphi[8][PBW];
  __shared__ R wc[8][NV][PCW];
  __shared__ R wA[8][TX];
  __shared__ R wsv[8][Q - 1][TX];

  const Dom& D = doms[t.x];
  if (k % D.N_phi) return;
  const int nx = D.nx, ny = D.ny, px = D.px, bcx = D.bc[0], bcy = D.bc[1];
  const long long pl = D.plane;
  const int x0 = t.y, ya = t.z, yb = t.w;
  const int w = min(TX, nx - x0);
  const unsigned np = n_phi(D, k - 1);
  const int ib = par(np), ob = ib ^ 1;
  GLOBAL const R* __restrict__ phi_in = gp<const R>(D.phi[qb(np)]);
  GLOBAL R* __restrict__ phi_out = gp<R>(D.phi[qb(np + 1)]);
  GLOBAL const SR* __restrict__ s_in = gp<const SR>(D.sphi[ib]);
  GLOBAL S* __restrict__ s_out = gp<S>(D.sphi[ob]);
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  GLOBAL const R* __restrict__ Up = D.has_U ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL const R* __restrict__ Tp = D.has_T ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;
  const PhaseConst<R> c = phase_const<R>(D);
  const R U0 = kc<R>(D, K_U0), T0 = kc<R>(D, K_T0);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;

  auto put_phi = [&](const YPhaseIn<R, S, Q>& in, int r0) {   // rows r0 + 1 .. r0 + 4
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int cc = tid + 256 * i;
      if (cc < 4 * PBW) wphi[(r0 + 1 + cc / PBW) & 7][cc % PBW] = in.phi[i];
    }
  };
  // collide rows r0 .. r0 + 3 (phase-field rows r0 - 1 .. r0 + 4 in LDS)
  auto collide = [&](const YPhaseIn<R, S, Q>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int col, row;
      if (!ym_cell64(i, tx, ty, tid, w, r0, col, row)) continue;
      if (resolve(x0 - 1 + col, nx, bcx) < 0 || resolve(row, ny, bcy) < 0) continue;   // beyond a wall
      const R* rm = wphi[(row - 1) & 7];
      const R* r0p = wphi[row & 7];
      const R* rp = wphi[(row + 1) & 7];
      R gx_, gy_;
      iso_grad_rows(rm, r0p, rp, col + 1, gx_, gy_);
      R sv[Q - 1];
#pragma unroll
      for (int q = 0; q < Q - 1; ++q) sv[q] = cvt_raw(in.s[i][q], (S*)nullptr);
      R jx, jy;
      if constexpr (Q == 5) {
        jx = sv[0] - sv[2];
        jy = sv[1] - sv[3];
      } else {
        jx = sv[0] - sv[2] + sv[4] - sv[5] - sv[6] + sv[7];
        jy = sv[1] - sv[3] + sv[4] + sv[5] - sv[6] - sv[7];
      }
      const R Uv = Up ? in.U[i] + U0 : R(0);
      const R Tv = Tp ? in.T[i] + T0 : c.theta_off;
      R dP, Kx, Ky, A, je[2];
      phase_collide(c, r0p[col + 1], gx_, gy_, jx, jy, Uv, Tv, dP, Kx, Ky, A, je);
      R(*cr)[PCW] = wc[row & 7];
      cr[0][col] = dP;
      cr[1][col] = Kx;
      cr[2][col] = Ky;
      if constexpr (Q == 9) {
        cr[3][col] = je[0];
        cr[4][col] = je[1];
      }
      if (i == 0) {
        wA[row & 7][tx] = A;
#pragma unroll
        for (int q = 0; q < Q - 1; ++q) wsv[row & 7][q][tx] = sv[q];
      }
    }
  };

  // prologue: phase-field rows ya - 4 .. ya + 1, collisions of ya - 3 .. ya
  YPhaseIn<R, S, Q> in0, in1;
  {
    YPhaseIn<R, S, Q> lo;
    ym_load_phase<R, S, Q>(nx, ny, px, bcx, bcy, x0, w, ya - 7, pl, tx, ty, tid, phi_in, s_in, Up, Tp, lo, false);
    ym_load_phase<R, S, Q>(nx, ny, px, bcx, bcy, x0, w, ya - 3, pl, tx, ty, tid, phi_in, s_in, Up, Tp, in1);
    put_phi(lo, ya - 7);   // rows ya - 6 .. ya - 3 (ya - 4 and ya - 3 are used)
    put_phi(in1, ya - 3);  // rows ya - 2 .. ya + 1
  }
  __syncthreads();
  collide(in1, ya - 3);
  ym_load_phase<R, S, Q>(nx, ny, px, bcx, bcy, x0, w, ya + 1, pl, tx, ty, tid, phi_in, s_in, Up, Tp, in0);
  __syncthreads();

  for (int y = ya; y < yb; y += 4) {
    // in0: collision inputs of rows y + 1 .. y + 4 and phase-field rows y + 2 .. y + 5
    // once the collision has consumed them, the loads for the next rows go
    // to the same registers and are in flight during the streaming
    put_phi(in0, y + 1);
    __syncthreads();
    collide(in0, y + 1);
    if (y + 4 < yb)
      ym_load_phase<R, S, Q>(nx, ny, px, bcx, bcy, x0, w, y + 5, pl, tx, ty, tid, phi_in, s_in, Up, Tp, in0);
    __syncthreads();
    const int gy = y + ty;
    // walls tested only on iterations whose rows or column touch one (the
    // test is uniform over the block)
    const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y == 0 || y + 4 >= ny));
    auto stream_rows = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
      if (tx < w && gy < yb) {
        // anisotropic pull streaming (Eq. 26) into the own site, in deviations
        const int gx = x0 + tx, lx = tx + 1;
        const R A = wA[gy & 7][tx], iA = rcp(A), oA = R(1) - A;
        const R phy = wphi[gy & 7][lx + 1];
        const R(*co)[PCW] = wc[gy & 7];
        const R dPo = co[0][lx];
        R sv[Q - 1];
#pragma unroll
        for (int q = 0; q < Q - 1; ++q) sv[q] = wsv[gy & 7][q][tx];
        R s0 = R(0);
#pragma unroll
        for (int q = 0; q < Q - 1; ++q) s0 -= sv[q];
        R dn[Q];
        dn[0] = (dPo * R(Lq::w(0)) - oA * s0) * iA;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
          const int ex = Lq::ex(q), ey = Lq::ey(q);
          const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                     (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
          R dpost;
          if (wall) {
            dpost = dPo * R(Lq::w(q)) - R(Lq::cK) * edot2(ex, ey, co[1][lx], co[2][lx]);
            if constexpr (Q == 9) dpost -= R(Lq::cJ(q)) * edot2(ex, ey, co[3][lx], co[4][lx]);
          } else {
            const R(*cu)[PCW] = wc[(gy - ey) & 7];
            const int ux = lx - ex;
            const R dphi = wphi[(gy - ey) & 7][ux + 1] - phy;
            dpost = (dphi + cu[0][ux]) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, cu[1][ux], cu[2][ux]);
            if constexpr (Q == 9) dpost += R(Lq::cJ(q)) * edot2(ex, ey, cu[3][ux], cu[4][ux]);
          }
          dn[q] = (dpost - oA * sv[q - 1]) * iA;
        }
        R dphin = dn[0];
#pragma unroll
        for (int q = 1; q < Q; ++q) dphin += dn[q];
        const unsigned o = (unsigned)gy * (unsigned)px + (unsigned)gx;
        sto(phi_out, o, phy + dphin);
#pragma unroll
        for (int q = 1; q < Q; ++q) sto(plane(s_out, (q - 1) * pl), o, dn[q] - dphin * R(Lq::w(q)));
      }
    };
    if (edge) stream_rows(std::true_type{});
    else stream_rows(std::false_type{});
    __syncthreads();
  }
}

// =================================================================== transfer
// Eq. (36)-(39): dphi = phi^{q+1} - phi^q; J = W0/(2 sqrt2) [1 + (1-k) U*]
// dphi n^{q+1}; dU = ([1 + (1-k)U*] dphi - 2 div J) / kfac(phi^{q+1});
// dT = rho_L L_h dphi / (2 rhoCp_eff(phi^{q+1})).  The compact divergence
// uses the D2Q9-weighted stencil; ghost J across a wall is the mirror image
// (normal component negated).  Instantaneous coupling adds dU to U and dT to
// T, each written to the next buffer (neighbours' U* and T* are read); the
// accumulated variant adds both to the pending planes.  Because
// the U and T states are stored as (chi, j), adding w_i d to every
// population is exactly adding d to chi.
template <class R, int TY>
__global__ __launch_bounds__(NTHR) void k_transfer(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                    unsigned k, Partial* __restrict__ part) {
  constexpr int RPT = TY / BY;
  constexpr int NS = RPT + 1;
  constexpr int BW = TX + 4, BH = TY + 4;
  constexpr int CW = TX + 2, CH = TY + 2;
  __shared__ R sphi[BH * BW];
  __shared__ R sJx[CH * CW], sJy[CH * CW];
  __shared__ R red[NTHR / 64];

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  if (k % D.N_phi) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px;
  const int x0 = t.y, y0 = t.z;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int bcx = D.bc[0], bcy = D.bc[1];
  GLOBAL const R* __restrict__ phi_old = gp<const R>(D.phi[qb(n_phi(D, k - 1))]);
  GLOBAL const R* __restrict__ phi_new = gp<const R>(D.phi[qb(n_phi(D, k))]);
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  GLOBAL const R* __restrict__ Uin = D.has_U ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL R* __restrict__ Uout = D.has_U ? gp<R>(D.U[qb(nU + 1)]) : nullptr;
  GLOBAL const R* __restrict__ Tin = D.has_T ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;
  GLOBAL R* __restrict__ Tout = D.has_T ? gp<R>(D.T[qb(n_T(D, k - 1) + 1)]) : nullptr;
  GLOBAL R* __restrict__ PU = gp<R>(D.PU);
  GLOBAL R* __restrict__ PT = gp<R>(D.PT);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R Uref = kc<R>(D, K_U0);   // the U plane holds U - U0
  const R cJ = kc<R>(D, K_CJ);
  const R cT = kc<R>(D, K_CT);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;

  if (!D.has_U) {
    // latent heat only: an own-site update, no stencil
    if (!D.has_T) return;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int gx = x0 + tx, gy = y0 + ty + r * BY;
      if (tx >= w || ty + r * BY >= h) continue;
      const unsigned o = gy * px + gx;
      const R pn = ldo(phi_new, o);
      const R dphi = pn - ldo(phi_old, o);
      const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
      const R dT = cT * dphi * rcp(R(2) * rc);
      if (D.accum)
        sto(PT, o, ldo(PT, o) + dT);
      else
        sto(Tout, o, ldo(Tin, o) + dT);
    }
    return;
  }

  // J on the owned sites and the ring (ghosts across walls mirror the wall
  // node with the normal component negated)
  int cl[NS], bi[NS];
  bool mxs[NS], mys[NS];
  R pold[NS], Us[NS], Tv[RPT];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    int lx, ly;
    cl[r] = -1;
    if (r < RPT) {
      lx = tx + 1;
      ly = ty + r * BY + 1;
      if (tx >= w || ly > h) continue;
    } else {
      if (!ring_cell(tid, w, h, lx, ly)) continue;
    }
    int rx = x0 - 1 + lx, ry = y0 - 1 + ly;
    bool mx = false, my = false;
    if (rx < 0 && bcx != BC_PER) { rx = 0; mx = true; }
    if (rx >= nx && bcx != BC_PER) { rx = nx - 1; mx = true; }
    if (ry < 0 && bcy != BC_PER) { ry = 0; my = true; }
    if (ry >= ny && bcy != BC_PER) { ry = ny - 1; my = true; }
    cl[r] = ly * CW + lx;
    bi[r] = (ry - (y0 - 2)) * BW + rx - (x0 - 2);
    mxs[r] = mx;
    mys[r] = my;
    const unsigned o = ghost(ry, ny, bcy) * px + ghost(rx, nx, bcx);
    pold[r] = ldo(phi_old, o);
    Us[r] = ldo(Uin, o);
    if (r < RPT && D.has_T) Tv[r] = D.accum ? ldo(PT, o) : ldo(Tin, o);
  }
  load_box2<R, BW, BH>(sphi, phi_new, px, x0, y0, nx, ny, bcx, bcy, tx, ty);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (cl[r] < 0) continue;
    const R* b = &sphi[bi[r]];
    R gxv, gyv;
    iso_grad(b, BW, gxv, gyv);
    const R gg = gxv * gxv + gyv * gyv;
    R Jx = R(0), Jy = R(0);
    if (gg >= R(GRAD_EPS2)) {
      const R ig = rsq(gg);
      const R a = cJ * (R(1) + omk * (Us[r] + Uref)) * (b[0] - pold[r]) * ig;
      Jx = -a * gxv;
      Jy = -a * gyv;
    }
    sJx[cl[r]] = mxs[r] ? -Jx : Jx;
    sJy[cl[r]] = mys[r] ? -Jy : Jy;
  }
  __syncthreads();

  R amax = R(0);
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (cl[r] < 0) continue;
    const int ci = cl[r];
    const unsigned o = (y0 + ty + r * BY) * px + x0 + tx;
    const R pn = sphi[bi[r]];
    const R dphi = pn - pold[r];
    const R* jx = &sJx[ci];
    const R* jy = &sJy[ci];
    const R div = (jx[1] - jx[-1]) * R(1.0 / 3.0) +
                  (jx[CW + 1] - jx[CW - 1] - jx[-CW - 1] + jx[-CW + 1]) * R(1.0 / 12.0) +
                  (jy[CW] - jy[-CW]) * R(1.0 / 3.0) +
                  (jy[CW + 1] + jy[CW - 1] - jy[-CW - 1] - jy[-CW + 1]) * R(1.0 / 12.0);
    const R dU = ((R(1) + omk * (Us[r] + Uref)) * dphi - R(2) * div) * rcp(opk - omk * pn);
    amax = fmax(amax, fabs(dU));
    if (D.accum)
      sto(PU, o, ldo(PU, o) + dU);
    else
      sto(Uout, o, Us[r] + dU);
    if (D.has_T) {
      const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
      const R dT = cT * dphi * rcp(R(2) * rc);
      if (D.accum)
        sto(PT, o, Tv[r] + dT);
      else
        sto(Tout, o, Tv[r] + dT);
    }
  }
  if (part) {
    // block max of |dU| (wavefront reduction, then across the 4 wavefronts)
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      part[t.w].S_phi = double(m);
      if (!D.accum) part[t.w].J_U = double(m);
    }
  }
}

// raw loads of the marching transfer: J inputs of rows r0 .. r0 + 3 (phi^q
// and U* at the column and ring cells, ghosted: beyond a wall, the
// boundary node) and phi^{q+1} rows r0 + 1 .. r0 + 4
template <class R>
struct YTrIn {
  R po[2], U[2];
  R phi[2];
};
template <class R>
__device__ __forceinline__ void ym_load_tr(int nx, int ny, int px, int bcx, int bcy, int x0, int w, int r0, int tx,
                                           int ty, int tid, GLOBAL const R* pn, GLOBAL const R* po,
                                           GLOBAL const R* Uin, YTrIn<R>& in, bool inputs = true) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!inputs) break;
    int col, row;
    if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
    const unsigned o = (unsigned)ghost(row, ny, bcy) * (unsigned)px + (unsigned)ghost(x0 - 1 + col, nx, bcx);
    in.po[i] = ldo(po, o);
    in.U[i] = ldo(Uin, o);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int cc = tid + 256 * i;
    if (cc < 4 * YBW) {
      const int gx = ghost(x0 - 2 + cc % YBW, nx, bcx), gy = ghost(r0 + 1 + cc / YBW, ny, bcy);
      in.phi[i] = ldo(pn, (unsigned)gy * (unsigned)px + (unsigned)gx);
    }
  }
}
// the own site of a row: phi^q, U*, T before the injection (or its pending
// plane), and phi^{q+1} when there is no U (and so no window)
template <class R>
struct YTrOwn {
  R po, U, T, pn;
};
template <class R>
__device__ __forceinline__ void ym_load_own(int ny, int px, int x0, int w, int row, int tx, bool hasU,
                                            GLOBAL const R* pn, GLOBAL const R* po, GLOBAL const R* Uin,
                                            GLOBAL const R* Tsrc, YTrOwn<R>& m) {
  if (tx < 1 || tx > w || row < 0 || row >= ny) return;
  const unsigned o = (unsigned)row * (unsigned)px + (unsigned)(x0 + tx - 1);
  m.po = ldo(po, o);
  if (hasU) m.U = ldo(Uin, o);
  else m.pn = ldo(pn, o);
  if (Tsrc) m.T = ldo(Tsrc, o);
}

// phase-step transfer (Eq. 36-39) marching up a column: J on the rows
// ahead (column plus ring; beyond a wall, the boundary node's J with the
// normal component negated), then the compact divergence, dU, dT and the
// injection on the current rows.  The largest |dU| of the run goes to its
// slot of the per-run maxima, where the diagnostics reduce it.
template <class R>
__device__ __forceinline__ void k_transfer_ym_run(const Dom* __restrict__ doms, const int4 t, unsigned k,
                                                  double2* __restrict__ rmax) {
  __shared__ R wphi[8][YBW];
  __shared__ R wJx[8][YCW], wJy[8][YCW];
  __shared__ R red[NTHR / 64];

  const Dom& D = doms[t.x];
  if (k % D.N_phi) return;
  const int nx = D.nx, ny = D.ny, px = D.px, bcx = D.bc[0], bcy = D.bc[1];
  const int x0 = t.y, ya = t.z, yb = t.w;
  const int w = min(YOW, nx - x0);
  GLOBAL const R* __restrict__ phi_old = gp<const R>(D.phi[qb(n_phi(D, k - 1))]);
  GLOBAL const R* __restrict__ phi_new = gp<const R>(D.phi[qb(n_phi(D, k))]);
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  const bool hasU = D.has_U, hasT = D.has_T, accum = D.accum;
  GLOBAL const R* __restrict__ Uin = hasU ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL R* __restrict__ Uout = hasU ? gp<R>(D.U[qb(nU + 1)]) : nullptr;
  GLOBAL R* __restrict__ Tout = hasT ? gp<R>(D.T[qb(n_T(D, k - 1) + 1)]) : nullptr;
  GLOBAL R* __restrict__ PU = gp<R>(D.PU);
  GLOBAL R* __restrict__ PT = gp<R>(D.PT);
  // T before the injection: the pending plane (accumulated coupling) or T
  GLOBAL const R* __restrict__ Tsrc = hasT ? (accum ? (GLOBAL const R*)PT : gp<const R>(D.T[qb(n_T(D, k - 1))]))
                                           : nullptr;
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R Uref = kc<R>(D, K_U0);   // the U plane holds U - U0
  const R cJ = kc<R>(D, K_CJ);
  const R cT = kc<R>(D, K_CT);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;

  auto put_phi = [&](const YTrIn<R>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int cc = tid + 256 * i;
      if (cc < 4 * YBW) wphi[(r0 + 1 + cc / YBW) & 7][cc % YBW] = in.phi[i];
    }
  };
  // J of rows r0 .. r0 + 3 (phi^{q+1} rows r0 - 1 .. r0 + 4 in LDS)
  auto flux = [&](const YTrIn<R>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int col, row;
      if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
      int rx = x0 - 1 + col, ry = row;
      bool mx = false, my = false;
      if (rx < 0 && bcx != BC_PER) { rx = 0; mx = true; }
      if (rx >= nx && bcx != BC_PER) { rx = nx - 1; mx = true; }
      if (ry < 0 && bcy != BC_PER) { ry = 0; my = true; }
      if (ry >= ny && bcy != BC_PER) { ry = ny - 1; my = true; }
      const int bcol = rx - (x0 - 2);   // window column of the (boundary) node
      R gxv, gyv;
      iso_grad_rows(wphi[(ry - 1) & 7], wphi[ry & 7], wphi[(ry + 1) & 7], bcol, gxv, gyv);
      const R gg = gxv * gxv + gyv * gyv;
      R Jx = R(0), Jy = R(0);
      if (gg >= R(GRAD_EPS2)) {
        const R ig = rsq(gg);
        const R a = cJ * (R(1) + omk * (in.U[i] + Uref)) * (wphi[ry & 7][bcol] - in.po[i]) * ig;
        Jx = -a * gxv;
        Jy = -a * gyv;
      }
      wJx[row & 7][col] = mx ? -Jx : Jx;
      wJy[row & 7][col] = my ? -Jy : Jy;
    }
  };

  R amax = R(0);
  YTrIn<R> in0;
  YTrOwn<R> own;
  // own sites of rows ya .. ya + 3; with U, phi^{q+1} rows ya - 6 .. ya + 1
  // and J of rows ya - 3 .. ya
  ym_load_own(ny, px, x0, w, ya + ty, tx, hasU, phi_new, phi_old, Uin, Tsrc, own);
  if (hasU) {
    YTrIn<R> lo, mid;
    ym_load_tr(nx, ny, px, bcx, bcy, x0, w, ya - 7, tx, ty, tid, phi_new, phi_old, Uin, lo, false);
    ym_load_tr(nx, ny, px, bcx, bcy, x0, w, ya - 3, tx, ty, tid, phi_new, phi_old, Uin, mid);
    put_phi(lo, ya - 7);
    put_phi(mid, ya - 3);
    __syncthreads();
    flux(mid, ya - 3);
    ym_load_tr(nx, ny, px, bcx, bcy, x0, w, ya + 1, tx, ty, tid, phi_new, phi_old, Uin, in0);
  }
  __syncthreads();

  for (int y = ya; y < yb; y += 4) {
    // in0: J inputs of rows y + 1 .. y + 4, phi^{q+1} rows y + 2 .. y + 5;
    // own: the own site of row y + ty
    if (hasU) put_phi(in0, y + 1);
    const YTrIn<R> cur = in0;
    const YTrOwn<R> me = own;
    if (y + 4 < yb) {   // prefetch for the next rows
      if (hasU) ym_load_tr(nx, ny, px, bcx, bcy, x0, w, y + 5, tx, ty, tid, phi_new, phi_old, Uin, in0);
      ym_load_own(ny, px, x0, w, y + 4 + ty, tx, hasU, phi_new, phi_old, Uin, Tsrc, own);
    }
    __syncthreads();
    if (hasU) flux(cur, y + 1);
    __syncthreads();
    const int gy = y + ty;
    if (tx >= 1 && tx <= w && gy < yb) {
      const int gx = x0 + tx - 1, lx = tx;
      const unsigned o = (unsigned)gy * (unsigned)px + (unsigned)gx;
      const R pn = hasU ? wphi[gy & 7][lx + 1] : me.pn;
      const R dphi = pn - me.po;
      if (hasU) {
        const int rm = (gy - 1) & 7, r0 = gy & 7, rp = (gy + 1) & 7;
        const R div = (wJx[r0][lx + 1] - wJx[r0][lx - 1]) * R(1.0 / 3.0) +
                      (wJx[rp][lx + 1] - wJx[rp][lx - 1] - wJx[rm][lx - 1] + wJx[rm][lx + 1]) * R(1.0 / 12.0) +
                      (wJy[rp][lx] - wJy[rm][lx]) * R(1.0 / 3.0) +
                      (wJy[rp][lx + 1] + wJy[rp][lx - 1] - wJy[rm][lx - 1] - wJy[rm][lx + 1]) * R(1.0 / 12.0);
        const R Us = me.U;
        const R dU = ((R(1) + omk * (Us + Uref)) * dphi - R(2) * div) * rcp(opk - omk * pn);
        amax = fmax(amax, fabs(dU));
        if (accum)
          sto(PU, o, ldo(PU, o) + dU);
        else
          sto(Uout, o, Us + dU);
      }
      if (hasT) {
        const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
        const R dT = cT * dphi * rcp(R(2) * rc);
        if (accum)
          sto(PT, o, me.T + dT);
        else
          sto(Tout, o, me.T + dT);
      }
    }
    __syncthreads();
  }
  if (rmax && hasU) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      double2& P = rmax[ym_run(D, x0, ya)];
      P.x = double(m);
      if (!accum) P.y = double(m);
    }
  }
}

// =================================================================== deferred transfer + phase
// The transfer of phase step k - 1 fused into the phase kernel of step k,
// for steps with no transport in between.  The transfer needs phi^{k-1} two
// sites away (J at a site takes the gradient of phi^{k-1}, the divergence
// at a collision cell the J of its neighbours), so the block reads phi^{k-1}
// on the tile plus three rings, computes J on the tile plus two rings and
// U*, T* = the transferred U, T on the tile plus one ring, where the phase
// collision uses them, and writes them on the tile.  Only loads and the
// cheap transfer arithmetic are repeated on the rings, no collisions, and
// the transfer's own launch disappears.  D2Q5, instantaneous coupling.
// The transfer's old phase field phi^{k-2}, read on two rings, sits in a
// buffer that this step's output does not use (four phase buffers), so
// neighbouring blocks never overwrite it.  Bitwise identical to the two
// separate kernels.
template <class R, class S, int TY>
__global__ __launch_bounds__(NTHR) void k_dtr_phase(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                     unsigned k, Partial* __restrict__ part) {
  constexpr int W3 = TX + 6, H3 = TY + 6;   // phi^{k-1} box
  constexpr int W2 = TX + 4, H2 = TY + 4;   // J
  constexpr int W1 = TX + 2, H1 = TY + 2;   // transferred U, T and the collisions
  constexpr int N3 = W3 * H3, N2 = W2 * H2, N1 = W1 * H1;
  constexpr int C2 = (N2 + NTHR - 1) / NTHR;
  constexpr int RPT = TY / BY, NS = RPT + 1;
  __shared__ R sq[N3];
  __shared__ R sJx[N2], sJy[N2];
  __shared__ R cP[N1], cKx[N1], cKy[N1];
  __shared__ R red[NTHR / 64];

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  if (k % D.N_phi) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px, pl = (int)D.plane;
  const int x0 = t.y, y0 = t.z;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int bcx = D.bc[0], bcy = D.bc[1];
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;
  const unsigned kt = k - 1;   // the transfer's step
  // transfer of step kt: phi^{kt-1} -> phi^{kt}; U, T of before -> after
  GLOBAL const R* __restrict__ phi_old = gp<const R>(D.phi[qb(n_phi(D, kt - 1))]);
  const unsigned np = n_phi(D, kt);
  const int ib = par(np), ob = ib ^ 1;
  GLOBAL const R* __restrict__ phi_in = gp<const R>(D.phi[qb(np)]);   // phi^{kt}: the transfer's new, the phase's input
  GLOBAL R* __restrict__ phi_out = gp<R>(D.phi[qb(np + 1)]);
  GLOBAL const S* __restrict__ s_in = gp<const S>(D.sphi[ib]);
  GLOBAL S* __restrict__ s_out = gp<S>(D.sphi[ob]);
  const unsigned nU = (kt - 1) / D.N_phi + (kt - 1) / D.N_U;
  GLOBAL const R* __restrict__ Uin = D.has_U ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL R* __restrict__ Uout = D.has_U ? gp<R>(D.U[qb(nU + 1)]) : nullptr;
  GLOBAL const R* __restrict__ Tin = D.has_T ? gp<const R>(D.T[qb(n_T(D, kt - 1))]) : nullptr;
  GLOBAL R* __restrict__ Tout = D.has_T ? gp<R>(D.T[qb(n_T(D, kt - 1) + 1)]) : nullptr;
  const PhaseConst<R> c = phase_const<R>(D);
  const R Uref = kc<R>(D, K_U0), Tref = kc<R>(D, K_T0);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R cJ = kc<R>(D, K_CJ), cT = kc<R>(D, K_CT);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  // raw coordinate -> position of the node whose values it takes in a
  // region of ring r (walls clamp, periodic axes keep the raw position)
  auto posx = [&](int g, int r) { return (wx ? min(max(g, 0), nx - 1) : g) - (x0 - r); };
  auto posy = [&](int g, int r) { return (wy ? min(max(g, 0), ny - 1) : g) - (y0 - r); };

  // ---- loads: phi^{kt} box; J inputs on ring 2; transfer and collision inputs on ring 1
  for (int i = tid; i < N3; i += NTHR)
    sq[i] = ldo(phi_in, (unsigned)(ghost(y0 - 3 + i / W3, ny, bcy) * px + ghost(x0 - 3 + i % W3, nx, bcx)));
  R jpo[C2], jU[C2];
#pragma unroll
  for (int j = 0; j < C2; ++j) {
    const int i = tid + j * NTHR;
    if (i >= N2) continue;
    const unsigned o = (unsigned)(ghost(y0 - 2 + i / W2, ny, bcy) * px + ghost(x0 - 2 + i % W2, nx, bcx));
    jpo[j] = ldo(phi_old, o);
    if (Uin) jU[j] = ldo(Uin, o);
  }
  // cells of this thread in the collision box (tile plus one ring): RPT
  // owned sites, then at most one ring cell (beyond a wall: none, never
  // pulled from), so the streaming below runs on every lane
  int cl[NS], bq[NS], ji[NS];   // collision-box, phi-box and J-box indices
  unsigned oc[NS];
  R sv[NS][4], cpo[NS], cU[NS], cT_[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    int lx, ly, gx, gy;
    cl[r] = -1;
    if (r < RPT) {
      lx = tx + 1;
      ly = ty + r * BY + 1;
      if (tx >= w || ly > h) continue;
      gx = x0 + tx;
      gy = y0 + ly - 1;
    } else {
      if (!ring_cell(tid, w, h, lx, ly)) continue;
      gx = resolve(x0 - 1 + lx, nx, bcx);
      gy = resolve(y0 - 1 + ly, ny, bcy);
      if (gx < 0 || gy < 0) continue;
    }
    cl[r] = ly * W1 + lx;
    bq[r] = (ly + 2) * W3 + lx + 2;
    ji[r] = (ly + 1) * W2 + lx + 1;
    const unsigned o = (unsigned)(gy * px + gx);
    oc[r] = o;
#pragma unroll
    for (int q = 0; q < 4; ++q) sv[r][q] = ldo(plane(s_in, q * pl), o);
    cpo[r] = ldo(phi_old, o);
    if (Uin) cU[r] = ldo(Uin, o);
    if (Tin) cT_[r] = ldo(Tin, o);
  }
  __syncthreads();

  // ---- J of step kt on ring 2 (beyond a wall: the clamped node's J with
  // its normal component negated), as the transfer kernel computes it
  if (Uin) {
#pragma unroll
    for (int j = 0; j < C2; ++j) {
      const int i = tid + j * NTHR;
      if (i >= N2) continue;
      const int gx = x0 - 2 + i % W2, gy = y0 - 2 + i / W2;
      const bool mx = wx && (gx < 0 || gx >= nx), my = wy && (gy < 0 || gy >= ny);
      const R* b = &sq[(posy(gy, 3)) * W3 + posx(gx, 3)];
      R gxv, gyv;
      iso_grad(b, W3, gxv, gyv);
      const R gg = gxv * gxv + gyv * gyv;
      R Jx = R(0), Jy = R(0);
      if (gg >= R(GRAD_EPS2)) {
        const R ig = rsq(gg);
        const R a = cJ * (R(1) + omk * (jU[j] + Uref)) * (b[0] - jpo[j]) * ig;
        Jx = -a * gxv;
        Jy = -a * gyv;
      }
      sJx[i] = mx ? -Jx : Jx;
      sJy[i] = my ? -Jy : Jy;
    }
  }
  __syncthreads();

  // ---- transferred U and T at the collision cells (stored on the owned
  // sites), then the phase collision there
  R amax = R(0), Aown[RPT];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (cl[r] < 0) continue;
    const bool own = r < RPT;
    const R* b = &sq[bq[r]];
    const R pn = b[0];
    const R dphi = pn - cpo[r];
    R Ust = R(0), Tst = R(0);
    if (Uin) {
      const R* jx = &sJx[ji[r]];
      const R* jy = &sJy[ji[r]];
      const R div = (jx[1] - jx[-1]) * R(1.0 / 3.0) +
                    (jx[W2 + 1] - jx[W2 - 1] - jx[-W2 - 1] + jx[-W2 + 1]) * R(1.0 / 12.0) +
                    (jy[W2] - jy[-W2]) * R(1.0 / 3.0) +
                    (jy[W2 + 1] + jy[W2 - 1] - jy[-W2 - 1] - jy[-W2 + 1]) * R(1.0 / 12.0);
      const R dU = ((R(1) + omk * (cU[r] + Uref)) * dphi - R(2) * div) * rcp(opk - omk * pn);
      Ust = cU[r] + dU;
      if (own) {
        amax = fmax(amax, fabs(dU));
        sto(Uout, oc[r], Ust);
      }
    }
    if (Tin) {
      const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
      const R dT = cT * dphi * rcp(R(2) * rc);
      Tst = cT_[r] + dT;
      if (own) sto(Tout, oc[r], Tst);
    }
    // the phase collision of step k with the transferred U and T
    R gxv, gyv;
    iso_grad(b, W3, gxv, gyv);
    const R Uv = Uin ? Ust + Uref : R(0);
    const R Tv = Tin ? Tst + Tref : c.theta_off;
    R dP, Kx, Ky, A;
    phase_collide(c, pn, gxv, gyv, sv[r][0] - sv[r][2], sv[r][1] - sv[r][3], Uv, Tv, dP, Kx, Ky, A);
    cP[cl[r]] = dP;
    cKx[cl[r]] = Kx;
    cKy[cl[r]] = Ky;
    if (own) Aown[r] = A;
  }
  __syncthreads();

  // ---- anisotropic pull streaming (Eq. 26) of the tile, in deviations
  const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y0 == 0 || y0 + h >= ny));
  auto stream = [&](auto edge_c) {
    constexpr bool EDGE = decltype(edge_c)::value;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (cl[r] < 0) continue;
      const int i = cl[r];
      const int gx = x0 + tx, gy = y0 + ty + r * BY;
      const R A = Aown[r], iA = rcp(A), oA = R(1) - A;
      const int bc = bq[r];
      const R phy = sq[bc];
      const R dPo = cP[i];
      R s0 = R(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) s0 -= sv[r][q];
      R dn[5];
      dn[0] = (dPo * R(1.0 / 3.0) - oA * s0) * iA;
#pragma unroll
      for (int q = 1; q < 5; ++q) {
        const int ex = EX5(q), ey = EY5(q);
        const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                   (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
        R dpost;
        if (wall) {
          dpost = dPo * R(1.0 / 6.0) - R(0.5) * edot2(ex, ey, cKx[i], cKy[i]);
        } else {
          const int si = i - ey * W1 - ex;
          const R dphi = sq[bc - ey * W3 - ex] - phy;
          dpost = (dphi + cP[si]) * R(1.0 / 6.0) + R(0.5) * edot2(ex, ey, cKx[si], cKy[si]);
        }
        dn[q] = (dpost - oA * sv[r][q - 1]) * iA;
      }
      R dphin = dn[0];
#pragma unroll
      for (int q = 1; q < 5; ++q) dphin += dn[q];
      const unsigned o = oc[r];
      sto(phi_out, o, phy + dphin);
#pragma unroll
      for (int q = 1; q < 5; ++q) sto(plane(s_out, (q - 1) * pl), o, dn[q] - dphin * R(1.0 / 6.0));
    }
  };
  if (edge) stream(std::true_type{});
  else stream(std::false_type{});

  if (part && Uin) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      part[t.w].S_phi = double(m);
      part[t.w].J_U = double(m);
    }
  }
}

// =================================================================== fused phase + transfer
// One phase update and its transfer (Eq. 26, then Eq. 36-39) in a single
// pass over a 64 x TY tile.  The transfer at a site needs phi^{q+1} two
// sites away (the anti-trapping current J one site away, its normal from
// the gradient of phi^{q+1}), so the block streams phi^{q+1} on the tile
// plus a ring of two, which needs the collisions on the tile plus a ring of
// three and phi^q on the tile plus four.  The rings are recomputed per
// block: phi^{q+1} never leaves LDS before the transfer, and the transfer
// has no launch of its own.  Arithmetic per site is that of k_phase and
// k_transfer, in the same order, so the results are bitwise identical.
//
// Region coordinates: a cell (lx, ly) of a region of ring r maps to the raw
// position (x0 - r + lx, y0 - r + ly).  On periodic axes that wraps; on
// wall axes, raw positions beyond the wall take the values of the clamped
// interior node (the even mirror about the half-way wall that the separate
// kernels' stencils use), and collisions there are not needed (streaming
// bounces back from the node itself).
template <class R, class S, int TY>
__global__ __launch_bounds__(NTHR) void k_phase_tr(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                    unsigned k, Partial* __restrict__ part) {
  constexpr int W4 = TX + 8, H4 = TY + 8;   // phi^q box
  constexpr int W3 = TX + 6, H3 = TY + 6;   // collisions
  constexpr int W2 = TX + 4, H2 = TY + 4;   // streaming, phi^{q+1}
  constexpr int W1 = TX + 2, H1 = TY + 2;   // J
  constexpr int N4 = W4 * H4, N3 = W3 * H3, N2 = W2 * H2, N1 = W1 * H1;
  constexpr int C3 = (N3 + NTHR - 1) / NTHR;   // collision cells per thread
  __shared__ R sq[N4];
  __shared__ R cP[N3], cKx[N3], cKy[N3], cA[N3];
  __shared__ R sn[N2];
  __shared__ R sJx[N1], sJy[N1];
  __shared__ R red[NTHR / 64];

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  if (k % D.N_phi) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px, pl = (int)D.plane;
  const int x0 = t.y, y0 = t.z;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int bcx = D.bc[0], bcy = D.bc[1];
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;
  const unsigned np = n_phi(D, k - 1);
  const int ib = par(np), ob = ib ^ 1;
  GLOBAL const R* __restrict__ phi_in = gp<const R>(D.phi[qb(np)]);
  GLOBAL R* __restrict__ phi_out = gp<R>(D.phi[qb(np + 1)]);
  GLOBAL const S* __restrict__ s_in = gp<const S>(D.sphi[ib]);
  GLOBAL S* __restrict__ s_out = gp<S>(D.sphi[ob]);
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  GLOBAL const R* __restrict__ Up = D.has_U ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL R* __restrict__ Uout = D.has_U ? gp<R>(D.U[qb(nU + 1)]) : nullptr;
  GLOBAL const R* __restrict__ Tin = D.has_T ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;
  GLOBAL R* __restrict__ Tout = D.has_T ? gp<R>(D.T[qb(n_T(D, k - 1) + 1)]) : nullptr;
  GLOBAL R* __restrict__ PU = gp<R>(D.PU);
  GLOBAL R* __restrict__ PT = gp<R>(D.PT);

  const PhaseConst<R> c = phase_const<R>(D);
  const R Uref = kc<R>(D, K_U0), Tref = kc<R>(D, K_T0);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R cJ = kc<R>(D, K_CJ);
  const R cT = kc<R>(D, K_CT);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const int tid = threadIdx.y * TX + threadIdx.x;

  // raw coordinate -> node whose values it takes (wrap or clamp)
  auto nodex = [&](int g) { return ghost(g, nx, bcx); };
  auto nodey = [&](int g) { return ghost(g, ny, bcy); };
  // raw coordinate -> its position in a region of ring r, after clamping at walls
  auto posx = [&](int g, int r) { return (wx ? min(max(g, 0), nx - 1) : g) - (x0 - r); };
  auto posy = [&](int g, int r) { return (wy ? min(max(g, 0), ny - 1) : g) - (y0 - r); };

  // ---- global loads: the collision inputs of this thread's cells, phi^q box
  R sv[C3][4], Uv[C3], Tv[C3];
  bool live[C3];
#pragma unroll
  for (int j = 0; j < C3; ++j) {
    const int cidx = tid + j * NTHR;
    live[j] = false;
    if (cidx >= N3) continue;
    const int gx = x0 - 3 + cidx % W3, gy = y0 - 3 + cidx / W3;
    const int rx = resolve(gx, nx, bcx), ry = resolve(gy, ny, bcy);
    if (rx < 0 || ry < 0) continue;                    // beyond a wall: never pulled from
    live[j] = true;
    const unsigned o = ry * px + rx;
    sv[j][0] = ldo(s_in, o);
    sv[j][1] = ldo(plane(s_in, pl), o);
    sv[j][2] = ldo(plane(s_in, 2 * pl), o);
    sv[j][3] = ldo(plane(s_in, 3 * pl), o);
    Uv[j] = Up ? ldo(Up, o) + Uref : R(0);
    Tv[j] = Tin ? ldo(Tin, o) + Tref : c.theta_off;
  }
  for (int cidx = tid; cidx < N4; cidx += NTHR) {
    const int gx = x0 - 4 + cidx % W4, gy = y0 - 4 + cidx / W4;
    sq[cidx] = phi_in[nodey(gy) * px + nodex(gx)];
  }
  __syncthreads();

  // ---- collisions on the tile + 3 ring
#pragma unroll
  for (int j = 0; j < C3; ++j) {
    if (!live[j]) continue;
    const int cidx = tid + j * NTHR;
    const int lx = cidx % W3, ly = cidx / W3;
    const R* b = &sq[(ly + 1) * W4 + lx + 1];
    R gxv, gyv;
    iso_grad(b, W4, gxv, gyv);
    R dP, Kx, Ky, A;
    phase_collide(c, b[0], gxv, gyv, sv[j][0] - sv[j][2], sv[j][1] - sv[j][3], Uv[j], Tv[j], dP, Kx, Ky, A);
    cP[cidx] = dP;
    cKx[cidx] = Kx;
    cKy[cidx] = Ky;
    cA[cidx] = A;
  }
  __syncthreads();

  // ---- anisotropic streaming on the tile + 2 ring (deviation form)
  for (int cidx = tid; cidx < N2; cidx += NTHR) {
    const int lx = cidx % W2, ly = cidx / W2;
    const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
    const int rx = resolve(gx, nx, bcx), ry = resolve(gy, ny, bcy);
    if (rx < 0 || ry < 0) continue;                    // filled from the clamped node below
    const unsigned o = ry * px + rx;
    const R s1 = ldo(s_in, o), s2 = ldo(plane(s_in, pl), o), s3 = ldo(plane(s_in, 2 * pl), o), s4 = ldo(plane(s_in, 3 * pl), o);
    const int ci = (ly + 1) * W3 + lx + 1;             // this node in the collision region
    const int bq = (ly + 2) * W4 + lx + 2;             // this node in the phi^q box
    const R A = cA[ci], iA = rcp(A), oA = R(1) - A;
    const R phy = sq[bq];
    const R dPo = cP[ci], Kxo = cKx[ci], Kyo = cKy[ci];
    const R svq[4] = {s1, s2, s3, s4};
    const R s0 = -(s1 + s2 + s3 + s4);
    const bool bb[5] = {false, wx && rx == 0, wy && ry == 0, wx && rx == nx - 1, wy && ry == ny - 1};
    R dn[5];
    dn[0] = (dPo * R(1.0 / 3.0) - oA * s0) * iA;
#pragma unroll
    for (int q = 1; q < 5; ++q) {
      const int ex = EX5(q), ey = EY5(q);
      R dpost;
      if (bb[q]) {
        dpost = dPo * R(1.0 / 6.0) - R(0.5) * edot2(ex, ey, Kxo, Kyo);
      } else {
        const int si = ci - ey * W3 - ex;
        const R dphi = sq[bq - ey * W4 - ex] - phy;
        dpost = (dphi + cP[si]) * R(1.0 / 6.0) + R(0.5) * edot2(ex, ey, cKx[si], cKy[si]);
      }
      dn[q] = (dpost - oA * svq[q - 1]) * iA;
    }
    const R dphin = dn[0] + dn[1] + dn[2] + dn[3] + dn[4];
    const R pn = phy + dphin;
    sn[cidx] = pn;
    if (lx >= 2 && ly >= 2 && lx - 2 < w && ly - 2 < h) {   // the tile: write the new state
      sto(phi_out, o, pn);
      sto(s_out, o, dn[1] - dphin * R(1.0 / 6.0));
      sto(plane(s_out, pl), o, dn[2] - dphin * R(1.0 / 6.0));
      sto(plane(s_out, 2 * pl), o, dn[3] - dphin * R(1.0 / 6.0));
      sto(plane(s_out, 3 * pl), o, dn[4] - dphin * R(1.0 / 6.0));
    }
  }
  __syncthreads();
  if (wx || wy) {   // raw positions beyond a wall take phi^{q+1} of the clamped node
    for (int cidx = tid; cidx < N2; cidx += NTHR) {
      const int lx = cidx % W2, ly = cidx / W2;
      const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
      if (resolve(gx, nx, bcx) >= 0 && resolve(gy, ny, bcy) >= 0) continue;
      sn[cidx] = sn[posy(gy, 2) * W2 + posx(gx, 2)];
    }
    __syncthreads();
  }

  if (!D.has_U) {
    // latent heat only: an own-site update
    if (!D.has_T) return;
    for (int cidx = tid; cidx < TX * TY; cidx += NTHR) {
      const int lx = cidx % TX, ly = cidx / TX;
      if (lx >= w || ly >= h) continue;
      const unsigned o = (y0 + ly) * px + x0 + lx;
      const R pn = sn[(ly + 2) * W2 + lx + 2];
      const R dphi = pn - sq[(ly + 4) * W4 + lx + 4];
      const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
      const R dT = cT * dphi * rcp(R(2) * rc);
      if (D.accum)
        sto(PT, o, ldo(PT, o) + dT);
      else
        sto(Tout, o, ldo(Tin, o) + dT);
    }
    return;
  }

  // ---- anti-trapping current on the tile + 1 ring (Eq. 37); beyond a wall
  // the current of the clamped node with its normal component negated
  for (int cidx = tid; cidx < N1; cidx += NTHR) {
    const int lx = cidx % W1, ly = cidx / W1;
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    const bool mx = wx && (gx < 0 || gx >= nx), my = wy && (gy < 0 || gy >= ny);
    const int qx = posx(gx, 1), qy = posy(gy, 1);      // node position in the J region
    const R* b = &sn[(qy + 1) * W2 + qx + 1];
    R gxv, gyv;
    iso_grad(b, W2, gxv, gyv);
    const R gg = gxv * gxv + gyv * gyv;
    R Jx = R(0), Jy = R(0);
    if (gg >= R(GRAD_EPS2)) {
      const unsigned o = nodey(gy) * px + nodex(gx);
      const R ig = rsq(gg);
      const R pold = sq[(qy + 3) * W4 + qx + 3];
      const R a = cJ * (R(1) + omk * (ldo(Up, o) + Uref)) * (b[0] - pold) * ig;
      Jx = -a * gxv;
      Jy = -a * gyv;
    }
    sJx[cidx] = mx ? -Jx : Jx;
    sJy[cidx] = my ? -Jy : Jy;
  }
  __syncthreads();

  // ---- increments of Eq. (38) and the injection of Eq. (39) on the tile
  R amax = R(0);
  for (int cidx = tid; cidx < TX * TY; cidx += NTHR) {
    const int lx = cidx % TX, ly = cidx / TX;
    if (lx >= w || ly >= h) continue;
    const unsigned o = (y0 + ly) * px + x0 + lx;
    const R pn = sn[(ly + 2) * W2 + lx + 2];
    const R dphi = pn - sq[(ly + 4) * W4 + lx + 4];
    const R* jx = &sJx[(ly + 1) * W1 + lx + 1];
    const R* jy = &sJy[(ly + 1) * W1 + lx + 1];
    const R div = (jx[1] - jx[-1]) * R(1.0 / 3.0) +
                  (jx[W1 + 1] - jx[W1 - 1] - jx[-W1 - 1] + jx[-W1 + 1]) * R(1.0 / 12.0) +
                  (jy[W1] - jy[-W1]) * R(1.0 / 3.0) +
                  (jy[W1 + 1] + jy[W1 - 1] - jy[-W1 - 1] - jy[-W1 + 1]) * R(1.0 / 12.0);
    const R Us = ldo(Up, o);
    const R dU = ((R(1) + omk * (Us + Uref)) * dphi - R(2) * div) * rcp(opk - omk * pn);
    amax = fmax(amax, fabs(dU));
    if (D.accum)
      sto(PU, o, ldo(PU, o) + dU);
    else
      sto(Uout, o, Us + dU);
    if (D.has_T) {
      const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
      const R dT = cT * dphi * rcp(R(2) * rc);
      if (D.accum)
        sto(PT, o, ldo(PT, o) + dT);
      else
        sto(Tout, o, ldo(Tin, o) + dT);
    }
  }
  if (part) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (threadIdx.x == 0) red[threadIdx.y] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      part[t.w].S_phi = double(m);
      if (!D.accum) part[t.w].J_U = double(m);
    }
  }
}

// =================================================================== scalar transport
// One update of U (FIELD 0) or T (FIELD 1): Eq. (14) with Eq. (19)-(20),
// (23), (24) and the transport source of Eq. (35) (first terms of Eq. 8 and
// Eq. 12) with grad chi from Eq. (40) and grad phi* from the isotropic
// stencil; then the streaming of Eq. (25) with half-way bounce-back and the
// reconstruction of chi and j.  The accumulated-coupling variant injects the
// pending increments right after the transport.
template <class R, class S, int TY, int FIELD, int Q>
__global__ __launch_bounds__(NTHR) void k_scalar(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                  unsigned k, Partial* __restrict__ part) {
  using Lq = Lat2<Q>;
  constexpr int RPT = TY / BY;
  constexpr int NS = RPT + 1;
  constexpr int BW = TX + 4, BH = TY + 4;
  constexpr int CW = TX + 2, CH = TY + 2;
  __shared__ R sphi[BH * BW];
  __shared__ R sC[CH * CW], sP[CH * CW], sKx[CH * CW], sKy[CH * CW];
  constexpr int NJ = Q == 9 ? CH * CW : 1;
  __shared__ R sJx[NJ], sJy[NJ];   // D2Q9: j_eq of the collision
  __shared__ R red[NTHR / 64];

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  const int N = FIELD == 0 ? D.N_U : D.N_T;
  if (k % N) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px, pl = (int)D.plane;
  const int x0 = t.y, y0 = t.z;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int bcx = D.bc[0], bcy = D.bc[1];
  GLOBAL const R* __restrict__ cin;
  GLOBAL R* __restrict__ cout;
  GLOBAL const S* __restrict__ jin;
  GLOBAL S* __restrict__ jout;
  GLOBAL R* __restrict__ pend;
  if (FIELD == 0) {
    const unsigned nU = (D.accum ? 0u : k / D.N_phi) + (k - 1) / D.N_U;
    cin = gp<const R>(D.U[qb(nU)]);
    cout = gp<R>(D.U[qb(nU + 1)]);
    jin = gp<const S>(D.jU[par(n_jU(D, k - 1))]);
    jout = gp<S>(D.jU[par(n_jU(D, k))]);
    pend = gp<R>(D.PU);
  } else {
    cin = gp<const R>(D.T[qb(n_Ttr(D, k) + (k - 1) / D.N_T)]);
    cout = gp<R>(D.T[qb(n_Ttr(D, k) + k / D.N_T)]);
    jin = gp<const S>(D.jT[par(n_jT(D, k - 1))]);
    jout = gp<S>(D.jT[par(n_jT(D, k))]);
    pend = gp<R>(D.PT);
  }
  GLOBAL const R* __restrict__ phis = gp<const R>(D.phi[qb(n_phi(D, k))]);
  // velocity of the latest flow update (the flow of step k runs after U, T)
  GLOBAL const R* __restrict__ vel = D.has_F ? gp<const R>(D.vel[par(n_F(D, k - 1))]) : nullptr;
  const bool need_phi = FIELD == 0 || D.T_var;
  const R dt = kc<R>(D, FIELD == 0 ? K_DTU : K_DTT);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R DS = kc<R>(D, K_DS), DL = kc<R>(D, K_DL);
  const R hkS = kc<R>(D, K_HKS), hkL = kc<R>(D, K_HKL), hrcS = kc<R>(D, K_HRCS), hrcL = kc<R>(D, K_HRCL);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const R itau_const = rcp(R(3) * dt * kc<R>(D, K_ALPHAL) + R(0.5));
  const R cref = kc<R>(D, FIELD == 0 ? K_U0 : K_T0);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;

  int cl[NS], bi[NS];
  R chi[NS], jxv[NS], jyv[NS], uxv[NS], uyv[NS], pv[RPT];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    int lx, ly, gx, gy;
    cl[r] = -1;
    if (r < RPT) {
      lx = tx + 1;
      ly = ty + r * BY + 1;
      if (tx >= w || ly > h) continue;
      gx = x0 + tx;
      gy = y0 + ly - 1;
    } else {
      if (!ring_cell(tid, w, h, lx, ly)) continue;
      gx = resolve(x0 - 1 + lx, nx, bcx);
      gy = resolve(y0 - 1 + ly, ny, bcy);
      if (gx < 0 || gy < 0) continue;
    }
    cl[r] = ly * CW + lx;
    bi[r] = (ly + 1) * BW + lx + 1;
    const unsigned o = gy * px + gx;
    chi[r] = ldo(cin, o);
    jxv[r] = ldo(jin, o);
    jyv[r] = ldo(plane(jin, pl), o);
    uxv[r] = vel ? ldo(vel, o) : R(0);
    uyv[r] = vel ? ldo(plane(vel, pl), o) : R(0);
    if (r < RPT && D.accum) pv[r] = ldo(pend, o);
  }
  if (need_phi) load_box2<R, BW, BH>(sphi, phis, px, x0, y0, nx, ny, bcx, bcy, tx, ty);
  __syncthreads();

#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (cl[r] < 0) continue;
    const R* b = &sphi[bi[r]];
    const R ca = chi[r] + cref;   // the plane holds chi - chi_ref
    const R jex = ca * uxv[r] * dt, jey = ca * uyv[r] * dt;
    R itau, Qs = R(0);
    if (FIELD == 0) {
      const R phi = b[0];
      const R ikf = rcp(opk - omk * phi);
      const R coeff = ((R(1) + phi) * DS + (R(1) - phi) * DL) * ikf;            // Eq. (7)
      itau = rcp(R(3) * dt * coeff + R(0.5));
      const R gcx = -R(3) * itau * (jxv[r] - jex), gcy = -R(3) * itau * (jyv[r] - jey);  // Eq. (40)
      R gpx, gpy;
      iso_grad(b, BW, gpx, gpy);
      Qs = -omk * coeff * (gcx * gpx + gcy * gpy) * ikf;                         // Eq. (8), 1st term
    } else if (D.T_var) {
      const R phi = b[0];
      const R irc = rcp((R(1) + phi) * hrcS + (R(1) - phi) * hrcL);
      const R coeff = ((R(1) + phi) * hkS + (R(1) - phi) * hkL) * irc;          // Eq. (11)
      itau = rcp(R(3) * dt * coeff + R(0.5));
      const R gcx = -R(3) * itau * (jxv[r] - jex), gcy = -R(3) * itau * (jyv[r] - jey);
      R gpx, gpy;
      iso_grad(b, BW, gpx, gpy);
      Qs = (hrcS - hrcL) * irc * coeff * (gcx * gpx + gcy * gpy);               // Eq. (12), 1st term
    } else {
      itau = itau_const;
    }
    const R om = R(1) - itau;
    sC[cl[r]] = chi[r];
    sP[cl[r]] = dt * Qs;
    sKx[cl[r]] = jex + om * (jxv[r] - jex);
    sKy[cl[r]] = jey + om * (jyv[r] - jey);
    if constexpr (Q == 9) {
      sJx[cl[r]] = jex;
      sJy[cl[r]] = jey;
    }
  }
  __syncthreads();

  // pull streaming (Eq. 25) in deviations d_i = f_i - w_i chi(y).  Only
  // tiles on a wall test the upstream node of each direction; the test is
  // uniform over the block, so interior tiles run without those branches.
  R amax = R(0);
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;
  const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y0 == 0 || y0 + h >= ny));
  auto stream = [&](auto edge_c) {
    constexpr bool EDGE = decltype(edge_c)::value;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (cl[r] < 0) continue;
      const int ci = cl[r];
      const int gx = x0 + tx, gy = y0 + ty + r * BY;
      const R cy = sC[ci], dPo = sP[ci];
      R dq[Q];
      dq[0] = dPo * R(Lq::w(0));
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        const int ex = Lq::ex(q), ey = Lq::ey(q);
        // the upstream node gx - ex, gy - ey lies beyond a wall
        const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                   (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
        if (EDGE && FIELD == 1 && D.T_dirlow && ey > 0 && gy == 0) {
          // anti-bounce-back to T0 at the wall y = -1/2 (the plane holds T - T0)
          dq[q] = -(R(2) * cy + dPo) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, sKx[ci], sKy[ci]);
          if constexpr (Q == 9) dq[q] += R(Lq::cJ(q)) * edot2(ex, ey, sJx[ci], sJy[ci]);
        } else if (wall) {
          dq[q] = dPo * R(Lq::w(q)) - R(Lq::cK) * edot2(ex, ey, sKx[ci], sKy[ci]);
          if constexpr (Q == 9) dq[q] -= R(Lq::cJ(q)) * edot2(ex, ey, sJx[ci], sJy[ci]);
        } else {
          const int si = ci - ey * CW - ex;
          dq[q] = (sC[si] - cy + sP[si]) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, sKx[si], sKy[si]);
          if constexpr (Q == 9) dq[q] += R(Lq::cJ(q)) * edot2(ex, ey, sJx[si], sJy[si]);
        }
      }
      const unsigned o = gy * px + gx;
      R sum = dq[0];
#pragma unroll
      for (int q = 1; q < Q; ++q) sum += dq[q];
      R chin = cy + sum;
      if (D.accum) {
        chin += pv[r];
        sto(pend, o, R(0));
        amax = fmax(amax, fabs(pv[r]));
      }
      sto(cout, o, chin);
      R jx = R(0), jy = R(0);
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        if (Lq::ex(q) > 0) jx += dq[q];
        if (Lq::ex(q) < 0) jx -= dq[q];
        if (Lq::ey(q) > 0) jy += dq[q];
        if (Lq::ey(q) < 0) jy -= dq[q];
      }
      sto(jout, o, jx);
      sto(plane(jout, pl), o, jy);
    }
  };
  if (edge) stream(std::true_type{});
  else stream(std::false_type{});
  if (FIELD == 0 && D.accum && part) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      part[t.w].J_U = double(m);
    }
  }
}

// =================================================================== transfer + U transport
// The transfer of phase step k fused into the U transport of the same step
// (the U update is due at k): the transport's collisions need the
// transferred U* on the tile plus one ring, so, as in the deferred-transfer
// phase kernel, the block reads phi^k on the tile plus three rings and
// phi^{k-1}, U on two rings, computes J on two rings and U* (and T* on the
// owned sites) itself, then collides and streams U.  U* is not written: its
// only reader is this transport, and the transported U goes to the buffer
// after it.  The U planes have four buffers, so the U before the transfer,
// read on the rings, is never the buffer neighbouring blocks write.  D2Q5,
// instantaneous coupling.  Bitwise identical to the two separate kernels.
template <class R, class S, int TY>
__global__ __launch_bounds__(NTHR) void k_dtr_scalar(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                      unsigned k, Partial* __restrict__ part) {
  using Lq = Lat2<5>;
  constexpr int W3 = TX + 6, H3 = TY + 6;   // phi^k box
  constexpr int W2 = TX + 4, H2 = TY + 4;   // J
  constexpr int W1 = TX + 2, H1 = TY + 2;   // U* and the transport collisions
  constexpr int N3 = W3 * H3, N2 = W2 * H2, N1 = W1 * H1;
  constexpr int C2 = (N2 + NTHR - 1) / NTHR;
  constexpr int RPT = TY / BY, NS = RPT + 1;
  __shared__ R sq[N3];
  __shared__ R sJx[N2], sJy[N2];
  __shared__ R sC[N1], sP[N1], sKx[N1], sKy[N1];
  __shared__ R red[NTHR / 64];

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  if (k % D.N_U) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px, pl = (int)D.plane;
  const int x0 = t.y, y0 = t.z;
  const int w = min(TX, nx - x0), h = min(TY, ny - y0);
  const int bcx = D.bc[0], bcy = D.bc[1];
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;
  // transfer of step k: phi^{k-1} -> phi^k, U -> U*; then U* -> the transported U
  GLOBAL const R* __restrict__ phi_old = gp<const R>(D.phi[qb(n_phi(D, k - 1))]);
  GLOBAL const R* __restrict__ phi_new = gp<const R>(D.phi[qb(n_phi(D, k))]);
  const unsigned nU = (k - 1) / D.N_phi + (k - 1) / D.N_U;
  GLOBAL const R* __restrict__ Uin = gp<const R>(D.U[qb(nU)]);
  GLOBAL R* __restrict__ Uout = gp<R>(D.U[qb(nU + 2)]);
  GLOBAL const R* __restrict__ Tin = D.has_T ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;
  GLOBAL R* __restrict__ Tout = D.has_T ? gp<R>(D.T[qb(n_T(D, k - 1) + 1)]) : nullptr;
  GLOBAL const S* __restrict__ jin = gp<const S>(D.jU[par(n_jU(D, k - 1))]);
  GLOBAL S* __restrict__ jout = gp<S>(D.jU[par(n_jU(D, k))]);
  GLOBAL const R* __restrict__ vel = D.has_F ? gp<const R>(D.vel[par(n_F(D, k - 1))]) : nullptr;
  const R Uref = kc<R>(D, K_U0);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R cJ = kc<R>(D, K_CJ), cT = kc<R>(D, K_CT);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const R dt = kc<R>(D, K_DTU);
  const R DS = kc<R>(D, K_DS), DL = kc<R>(D, K_DL);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  // raw coordinate -> position of the node whose values it takes in a
  // region of ring r (walls clamp, periodic axes keep the raw position)
  auto posx = [&](int g, int r) { return (wx ? min(max(g, 0), nx - 1) : g) - (x0 - r); };
  auto posy = [&](int g, int r) { return (wy ? min(max(g, 0), ny - 1) : g) - (y0 - r); };

  // ---- loads: phi^k box; J inputs on ring 2; transfer and transport inputs
  // at the collision cells (RPT owned sites, then at most one ring cell)
  for (int i = tid; i < N3; i += NTHR)
    sq[i] = ldo(phi_new, (unsigned)(ghost(y0 - 3 + i / W3, ny, bcy) * px + ghost(x0 - 3 + i % W3, nx, bcx)));
  R jpo[C2], jU[C2];
#pragma unroll
  for (int j = 0; j < C2; ++j) {
    const int i = tid + j * NTHR;
    if (i >= N2) continue;
    const unsigned o = (unsigned)(ghost(y0 - 2 + i / W2, ny, bcy) * px + ghost(x0 - 2 + i % W2, nx, bcx));
    jpo[j] = ldo(phi_old, o);
    jU[j] = ldo(Uin, o);
  }
  int cl[NS], bq[NS], ji[NS];
  unsigned oc[NS];
  R cpo[NS], cU[NS], jxv[NS], jyv[NS], uxv[NS], uyv[NS], cT_[RPT];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    int lx, ly, gx, gy;
    cl[r] = -1;
    if (r < RPT) {
      lx = tx + 1;
      ly = ty + r * BY + 1;
      if (tx >= w || ly > h) continue;
      gx = x0 + tx;
      gy = y0 + ly - 1;
    } else {
      if (!ring_cell(tid, w, h, lx, ly)) continue;
      gx = resolve(x0 - 1 + lx, nx, bcx);
      gy = resolve(y0 - 1 + ly, ny, bcy);
      if (gx < 0 || gy < 0) continue;   // beyond a wall: never pulled from
    }
    cl[r] = ly * W1 + lx;
    bq[r] = (ly + 2) * W3 + lx + 2;
    ji[r] = (ly + 1) * W2 + lx + 1;
    const unsigned o = (unsigned)(gy * px + gx);
    oc[r] = o;
    cpo[r] = ldo(phi_old, o);
    cU[r] = ldo(Uin, o);
    jxv[r] = ldo(jin, o);
    jyv[r] = ldo(plane(jin, pl), o);
    uxv[r] = vel ? ldo(vel, o) : R(0);
    uyv[r] = vel ? ldo(plane(vel, pl), o) : R(0);
    if (r < RPT && Tin) cT_[r] = ldo(Tin, o);
  }
  __syncthreads();

  // ---- J of step k on ring 2 (beyond a wall: the clamped node's J with its
  // normal component negated), as the transfer kernel computes it
#pragma unroll
  for (int j = 0; j < C2; ++j) {
    const int i = tid + j * NTHR;
    if (i >= N2) continue;
    const int gx = x0 - 2 + i % W2, gy = y0 - 2 + i / W2;
    const bool mx = wx && (gx < 0 || gx >= nx), my = wy && (gy < 0 || gy >= ny);
    const R* b = &sq[(posy(gy, 3)) * W3 + posx(gx, 3)];
    R gxv, gyv;
    iso_grad(b, W3, gxv, gyv);
    const R gg = gxv * gxv + gyv * gyv;
    R Jx = R(0), Jy = R(0);
    if (gg >= R(GRAD_EPS2)) {
      const R ig = rsq(gg);
      const R a = cJ * (R(1) + omk * (jU[j] + Uref)) * (b[0] - jpo[j]) * ig;
      Jx = -a * gxv;
      Jy = -a * gyv;
    }
    sJx[i] = mx ? -Jx : Jx;
    sJy[i] = my ? -Jy : Jy;
  }
  __syncthreads();

  // ---- U* at the collision cells (T* on the owned sites), then the U
  // collision of Eq. (14) with the transport source, as the transport
  // kernel computes them
  R amax = R(0);
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    if (cl[r] < 0) continue;
    const bool own = r < RPT;
    const R* b = &sq[bq[r]];
    const R pn = b[0];
    const R dphi = pn - cpo[r];
    const R* jx = &sJx[ji[r]];
    const R* jy = &sJy[ji[r]];
    const R div = (jx[1] - jx[-1]) * R(1.0 / 3.0) +
                  (jx[W2 + 1] - jx[W2 - 1] - jx[-W2 - 1] + jx[-W2 + 1]) * R(1.0 / 12.0) +
                  (jy[W2] - jy[-W2]) * R(1.0 / 3.0) +
                  (jy[W2 + 1] + jy[W2 - 1] - jy[-W2 - 1] - jy[-W2 + 1]) * R(1.0 / 12.0);
    const R dU = ((R(1) + omk * (cU[r] + Uref)) * dphi - R(2) * div) * rcp(opk - omk * pn);
    const R chi = cU[r] + dU;
    if (own) {
      amax = fmax(amax, fabs(dU));
      if (Tin) {
        const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
        const R dT = cT * dphi * rcp(R(2) * rc);
        sto(Tout, oc[r], cT_[r] + dT);
      }
    }
    const R ca = chi + Uref;
    const R jex = ca * uxv[r] * dt, jey = ca * uyv[r] * dt;
    const R phi = pn;
    const R ikf = rcp(opk - omk * phi);
    const R coeff = ((R(1) + phi) * DS + (R(1) - phi) * DL) * ikf;
    const R itau = rcp(R(3) * dt * coeff + R(0.5));
    const R gcx = -R(3) * itau * (jxv[r] - jex), gcy = -R(3) * itau * (jyv[r] - jey);
    R gpx, gpy;
    iso_grad(b, W3, gpx, gpy);
    const R Qs = -omk * coeff * (gcx * gpx + gcy * gpy) * ikf;
    const R om = R(1) - itau;
    sC[cl[r]] = chi;
    sP[cl[r]] = dt * Qs;
    sKx[cl[r]] = jex + om * (jxv[r] - jex);
    sKy[cl[r]] = jey + om * (jyv[r] - jey);
  }
  __syncthreads();

  // ---- pull streaming (Eq. 25) of the tile in deviations
  const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y0 == 0 || y0 + h >= ny));
  auto stream = [&](auto edge_c) {
    constexpr bool EDGE = decltype(edge_c)::value;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if (cl[r] < 0) continue;
      const int ci = cl[r];
      const int gx = x0 + tx, gy = y0 + ty + r * BY;
      const R cy = sC[ci], dPo = sP[ci];
      R dq[5];
      dq[0] = dPo * R(Lq::w(0));
#pragma unroll
      for (int q = 1; q < 5; ++q) {
        const int ex = Lq::ex(q), ey = Lq::ey(q);
        const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                   (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
        if (wall) {
          dq[q] = dPo * R(Lq::w(q)) - R(Lq::cK) * edot2(ex, ey, sKx[ci], sKy[ci]);
        } else {
          const int si = ci - ey * W1 - ex;
          dq[q] = (sC[si] - cy + sP[si]) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, sKx[si], sKy[si]);
        }
      }
      const unsigned o = oc[r];
      R sum = dq[0];
#pragma unroll
      for (int q = 1; q < 5; ++q) sum += dq[q];
      const R chin = cy + sum;
      sto(Uout, o, chin);
      R jx = R(0), jy = R(0);
#pragma unroll
      for (int q = 1; q < 5; ++q) {
        if (Lq::ex(q) > 0) jx += dq[q];
        if (Lq::ex(q) < 0) jx -= dq[q];
        if (Lq::ey(q) > 0) jy += dq[q];
        if (Lq::ey(q) < 0) jy -= dq[q];
      }
      sto(jout, o, jx);
      sto(plane(jout, pl), o, jy);
    }
  };
  if (edge) stream(std::true_type{});
  else stream(std::false_type{});

  if (part) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      part[t.w].S_phi = double(m);
      part[t.w].J_U = double(m);
    }
  }
}

// raw loads of the marching scalar transport for the rows r0 .. r0 + 3:
// chi, j and the velocity at the column and ring cells (beyond a wall: no
// cell), the phase field rows r0 + 1 .. r0 + 4, and the own pending
// increment of row r0 - 1 + ty (the row streamed while these are collided)
template <class R, class S>
struct YScIn {
  R chi[2], u[2][2];
  typename RawT<S>::type j[2][2];
  R phi[2];
  R pend;
};
template <class R, class S>
__device__ __forceinline__ void ym_load_sc(int nx, int ny, int px, int bcx, int bcy, int x0, int w, int r0, int tx,
                                           int ty, int tid, long long pl, bool need_phi, GLOBAL const R* phis,
                                           GLOBAL const R* cin, GLOBAL const typename RawT<S>::type* jin,
                                           GLOBAL const R* vel, GLOBAL const R* pend, YScIn<R, S>& in,
                                           bool inputs = true) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!inputs) break;
    int col, row;
    if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
    const int gx = resolve(x0 - 1 + col, nx, bcx), gy = resolve(row, ny, bcy);
    if (gx < 0 || gy < 0) continue;
    const unsigned o = (unsigned)gy * (unsigned)px + (unsigned)gx;
    in.chi[i] = ldo(cin, o);
    in.j[i][0] = *at(jin, o);
    in.j[i][1] = *at(plane(jin, pl), o);
    if (vel) {
      in.u[i][0] = ldo(vel, o);
      in.u[i][1] = ldo(plane(vel, pl), o);
    }
  }
  if (need_phi) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int cc = tid + 256 * i;
      if (cc < 4 * YBW) {
        const int gx = ghost(x0 - 2 + cc % YBW, nx, bcx), gy = ghost(r0 + 1 + cc / YBW, ny, bcy);
        in.phi[i] = ldo(phis, (unsigned)gy * (unsigned)px + (unsigned)gx);
      }
    }
  }
  const int oy = r0 - 1 + ty;
  if (pend && inputs && tx >= 1 && tx <= w && oy >= 0 && oy < ny)
    in.pend = ldo(pend, (unsigned)oy * (unsigned)px + (unsigned)(x0 + tx - 1));
}

// scalar transport (U: FIELD 0, T: FIELD 1) marching up a column: the
// collision of Eq. (14) with the equilibrium of Eq. (19)-(20), tau of Eq.
// (7) or (11) and the source of Eq. (8) or (12) with grad chi from Eq. (40)
// on the rows ahead, then the pull streaming of Eq. (25) on the current
// rows.  With accumulated coupling the largest pending |dU| of the run goes
// to its slot of the per-run maxima.
template <class R, class S, int FIELD, int Q>
__device__ __forceinline__ void k_scalar_ym_run(const Dom* __restrict__ doms, const int4 t, unsigned k,
                                                double2* __restrict__ rmax) {
  using Lq = Lat2<Q>;
  using SR = typename RawT<S>::type;
  constexpr int NV = Q == 9 ? 6 : 4;   // chi, dt Q, Kx, Ky (and j_eq in D2Q9)
  __shared__ R wphi[8][YBW];
  __shared__ R wc[8][NV][YCW];
  __shared__ R red[NTHR / 64];

  const Dom& D = doms[t.x];
  const int N = FIELD == 0 ? D.N_U : D.N_T;
  if (k % N) return;
  const int nx = D.nx, ny = D.ny, px = D.px, bcx = D.bc[0], bcy = D.bc[1];
  const long long pl = D.plane;
  const int x0 = t.y, ya = t.z, yb = t.w;
  const int w = min(YOW, nx - x0);
  GLOBAL const R* __restrict__ cin;
  GLOBAL R* __restrict__ cout;
  GLOBAL const SR* __restrict__ jin;
  GLOBAL S* __restrict__ jout;
  GLOBAL R* __restrict__ pend;
  if (FIELD == 0) {
    const unsigned nU = (D.accum ? 0u : k / D.N_phi) + (k - 1) / D.N_U;
    cin = gp<const R>(D.U[qb(nU)]);
    cout = gp<R>(D.U[qb(nU + 1)]);
    jin = gp<const SR>(D.jU[par(n_jU(D, k - 1))]);
    jout = gp<S>(D.jU[par(n_jU(D, k))]);
    pend = gp<R>(D.PU);
  } else {
    cin = gp<const R>(D.T[qb(n_Ttr(D, k) + (k - 1) / D.N_T)]);
    cout = gp<R>(D.T[qb(n_Ttr(D, k) + k / D.N_T)]);
    jin = gp<const SR>(D.jT[par(n_jT(D, k - 1))]);
    jout = gp<S>(D.jT[par(n_jT(D, k))]);
    pend = gp<R>(D.PT);
  }
  GLOBAL const R* __restrict__ phis = gp<const R>(D.phi[qb(n_phi(D, k))]);
  GLOBAL const R* __restrict__ vel = D.has_F ? gp<const R>(D.vel[par(n_F(D, k - 1))]) : nullptr;
  const bool need_phi = FIELD == 0 || D.T_var;
  const bool accum = D.accum;
  GLOBAL const R* __restrict__ pend_in = accum ? (GLOBAL const R*)pend : nullptr;
  const R dt = kc<R>(D, FIELD == 0 ? K_DTU : K_DTT);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R DS = kc<R>(D, K_DS), DL = kc<R>(D, K_DL);
  const R hkS = kc<R>(D, K_HKS), hkL = kc<R>(D, K_HKL), hrcS = kc<R>(D, K_HRCS), hrcL = kc<R>(D, K_HRCL);
  const R itau_const = rcp(R(3) * dt * kc<R>(D, K_ALPHAL) + R(0.5));
  const R cref = kc<R>(D, FIELD == 0 ? K_U0 : K_T0);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;

  auto put_phi = [&](const YScIn<R, S>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int cc = tid + 256 * i;
      if (cc < 4 * YBW) wphi[(r0 + 1 + cc / YBW) & 7][cc % YBW] = in.phi[i];
    }
  };
  auto collide = [&](const YScIn<R, S>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int col, row;
      if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
      if (resolve(x0 - 1 + col, nx, bcx) < 0 || resolve(row, ny, bcy) < 0) continue;   // beyond a wall
      const R chi = in.chi[i];
      const R ca = chi + cref;   // the plane holds chi - chi_ref
      const R uxv = vel ? in.u[i][0] : R(0), uyv = vel ? in.u[i][1] : R(0);
      const R jxv = cvt_raw(in.j[i][0], (S*)nullptr), jyv = cvt_raw(in.j[i][1], (S*)nullptr);
      const R jex = ca * uxv * dt, jey = ca * uyv * dt;
      R itau, Qs = R(0);
      if (FIELD == 0) {
        const R* r0p = wphi[row & 7];
        const R phi = r0p[col + 1];
        const R ikf = rcp(opk - omk * phi);
        const R coeff = ((R(1) + phi) * DS + (R(1) - phi) * DL) * ikf;            // Eq. (7)
        itau = rcp(R(3) * dt * coeff + R(0.5));
        const R gcx = -R(3) * itau * (jxv - jex), gcy = -R(3) * itau * (jyv - jey);  // Eq. (40)
        R gpx, gpy;
        iso_grad_rows(wphi[(row - 1) & 7], r0p, wphi[(row + 1) & 7], col + 1, gpx, gpy);
        Qs = -omk * coeff * (gcx * gpx + gcy * gpy) * ikf;                         // Eq. (8), 1st term
      } else if (need_phi) {
        const R* r0p = wphi[row & 7];
        const R phi = r0p[col + 1];
        const R irc = rcp((R(1) + phi) * hrcS + (R(1) - phi) * hrcL);
        const R coeff = ((R(1) + phi) * hkS + (R(1) - phi) * hkL) * irc;          // Eq. (11)
        itau = rcp(R(3) * dt * coeff + R(0.5));
        const R gcx = -R(3) * itau * (jxv - jex), gcy = -R(3) * itau * (jyv - jey);
        R gpx, gpy;
        iso_grad_rows(wphi[(row - 1) & 7], r0p, wphi[(row + 1) & 7], col + 1, gpx, gpy);
        Qs = (hrcS - hrcL) * irc * coeff * (gcx * gpx + gcy * gpy);               // Eq. (12), 1st term
      } else {
        itau = itau_const;
      }
      const R om = R(1) - itau;
      R(*cr)[YCW] = wc[row & 7];
      cr[0][col] = chi;
      cr[1][col] = dt * Qs;
      cr[2][col] = jex + om * (jxv - jex);
      cr[3][col] = jey + om * (jyv - jey);
      if constexpr (Q == 9) {
        cr[4][col] = jex;
        cr[5][col] = jey;
      }
    }
  };

  R amax = R(0);
  YScIn<R, S> in0;
  {
    YScIn<R, S> lo, mid;
    if (need_phi) {
      ym_load_sc<R, S>(nx, ny, px, bcx, bcy, x0, w, ya - 7, tx, ty, tid, pl, true, phis, cin, jin, vel, nullptr, lo,
                       false);
      put_phi(lo, ya - 7);
    }
    ym_load_sc<R, S>(nx, ny, px, bcx, bcy, x0, w, ya - 3, tx, ty, tid, pl, need_phi, phis, cin, jin, vel, nullptr, mid);
    if (need_phi) put_phi(mid, ya - 3);
    __syncthreads();
    collide(mid, ya - 3);
    ym_load_sc<R, S>(nx, ny, px, bcx, bcy, x0, w, ya + 1, tx, ty, tid, pl, need_phi, phis, cin, jin, vel, pend_in,
                     in0);
  }
  __syncthreads();

  for (int y = ya; y < yb; y += 4) {
    // in0: inputs of rows y + 1 .. y + 4, phase field rows y + 2 .. y + 5,
    // own pending increment of row y + ty (in pcur)
    if (need_phi) put_phi(in0, y + 1);
    const YScIn<R, S> cur = in0;
    if (y + 4 < yb)
      ym_load_sc<R, S>(nx, ny, px, bcx, bcy, x0, w, y + 5, tx, ty, tid, pl, need_phi, phis, cin, jin, vel, pend_in,
                       in0);
    __syncthreads();
    collide(cur, y + 1);
    __syncthreads();
    const int gy = y + ty;
    // walls tested only on iterations whose rows or column touch one (the
    // test is uniform over the block)
    const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y == 0 || y + 4 >= ny));
    auto stream_rows = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
      if (tx >= 1 && tx <= w && gy < yb) {
        // pull streaming (Eq. 25) in deviations d_i = f_i - w_i chi(y)
        const int gx = x0 + tx - 1, lx = tx;
        const R(*co)[YCW] = wc[gy & 7];
        const R cy = co[0][lx], dPo = co[1][lx];
        R dq[Q];
        dq[0] = dPo * R(Lq::w(0));
#pragma unroll
        for (int q = 1; q < Q; ++q) {
          const int ex = Lq::ex(q), ey = Lq::ey(q);
          const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                     (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
          if (EDGE && FIELD == 1 && D.T_dirlow && ey > 0 && gy == 0) {
            // anti-bounce-back to T0 at the wall y = -1/2 (the plane holds T - T0)
            dq[q] = -(R(2) * cy + dPo) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, co[2][lx], co[3][lx]);
            if constexpr (Q == 9) dq[q] += R(Lq::cJ(q)) * edot2(ex, ey, co[4][lx], co[5][lx]);
          } else if (wall) {
            dq[q] = dPo * R(Lq::w(q)) - R(Lq::cK) * edot2(ex, ey, co[2][lx], co[3][lx]);
            if constexpr (Q == 9) dq[q] -= R(Lq::cJ(q)) * edot2(ex, ey, co[4][lx], co[5][lx]);
          } else {
            const R(*cu)[YCW] = wc[(gy - ey) & 7];
            const int ux = lx - ex;
            dq[q] = (cu[0][ux] - cy + cu[1][ux]) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, cu[2][ux], cu[3][ux]);
            if constexpr (Q == 9) dq[q] += R(Lq::cJ(q)) * edot2(ex, ey, cu[4][ux], cu[5][ux]);
          }
        }
        const unsigned o = (unsigned)gy * (unsigned)px + (unsigned)gx;
        R sum = dq[0];
#pragma unroll
        for (int q = 1; q < Q; ++q) sum += dq[q];
        R chin = cy + sum;
        if (accum) {
          chin += cur.pend;
          sto(pend, o, R(0));
          amax = fmax(amax, fabs(cur.pend));
        }
        sto(cout, o, chin);
        R jx = R(0), jy = R(0);
#pragma unroll
        for (int q = 1; q < Q; ++q) {
          if (Lq::ex(q) > 0) jx += dq[q];
          if (Lq::ex(q) < 0) jx -= dq[q];
          if (Lq::ey(q) > 0) jy += dq[q];
          if (Lq::ey(q) < 0) jy -= dq[q];
        }
        sto(jout, o, jx);
        sto(plane(jout, pl), o, jy);
      }
    };
    if (edge) stream_rows(std::true_type{});
    else stream_rows(std::false_type{});
    __syncthreads();
  }
  if (FIELD == 0 && accum && rmax) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      rmax[ym_run(D, x0, ya)].y = double(m);
    }
  }
}


// =================================================================== transfer + T transport, marching
// raw loads of the marching transfer + T transport for the rows r0 .. r0 + 3:
// the J inputs phi^q and U at the column and ring cells (ghosted: beyond a
// wall, the boundary node), and where the cell is a collision cell (not
// beyond a wall) T before the transfer, j_T and the velocity; then phi^{q+1}
// rows r0 + 1 .. r0 + 4
template <class R, class S>
struct YTsIn {
  R po[2], U[2], T[2], u[2][2];
  typename RawT<S>::type j[2][2];
  R phi[2];
};
template <class R, class S>
__device__ __forceinline__ void ym_load_ts(int nx, int ny, int px, int bcx, int bcy, int x0, int w, int r0, int tx,
                                           int ty, int tid, long long pl, GLOBAL const R* pn, GLOBAL const R* po,
                                           GLOBAL const R* Uin, GLOBAL const R* Tin,
                                           GLOBAL const typename RawT<S>::type* jin, GLOBAL const R* vel,
                                           YTsIn<R, S>& in, bool inputs = true) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!inputs) break;
    int col, row;
    if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
    const int rx = x0 - 1 + col;
    // inside the domain and across periodic edges the ghost and the
    // resolved node coincide
    const unsigned o = (unsigned)ghost(row, ny, bcy) * (unsigned)px + (unsigned)ghost(rx, nx, bcx);
    in.po[i] = ldo(po, o);
    if (Uin) in.U[i] = ldo(Uin, o);
    if (resolve(rx, nx, bcx) < 0 || resolve(row, ny, bcy) < 0) continue;
    in.T[i] = ldo(Tin, o);
    in.j[i][0] = *at(jin, o);
    in.j[i][1] = *at(plane(jin, pl), o);
    if (vel) {
      in.u[i][0] = ldo(vel, o);
      in.u[i][1] = ldo(plane(vel, pl), o);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int cc = tid + 256 * i;
    if (cc < 4 * YBW) {
      const int gx = ghost(x0 - 2 + cc % YBW, nx, bcx), gy = ghost(r0 + 1 + cc / YBW, ny, bcy);
      in.phi[i] = ldo(pn, (unsigned)gy * (unsigned)px + (unsigned)gx);
    }
  }
}

// The transfer of phase step k fused into the T transport of the same step,
// marching up a column (a step at which both are due, instantaneous
// coupling).  On the rows ahead: J (as the marching transfer), and at the
// collision cells T* = T + dT of the transfer and the T collision with it;
// on the current rows: U* = U + dU (written) and the T streaming.  T* is
// not written: its only reader is this transport, and the transported T
// goes to the buffer after it.  The T planes have four buffers, so the T
// before the transfer, read on the rings, is never the buffer neighbouring
// blocks write.  The U transport of the step runs after this kernel.
// Bitwise identical to the two separate kernels.
template <class R, class S, int Q>
__device__ __forceinline__ void k_tr_scalar_ym_run(const Dom* __restrict__ doms, const int4 t, unsigned k,
                                                   double2* __restrict__ rmax) {
  using Lq = Lat2<Q>;
  using SR = typename RawT<S>::type;
  constexpr int NV = Q == 9 ? 6 : 4;   // chi, dt Q, Kx, Ky (and j_eq in D2Q9)
  __shared__ R wphi[8][YBW];
  __shared__ R wJx[8][YCW], wJy[8][YCW];
  __shared__ R wc[8][NV][YCW];
  __shared__ R red[NTHR / 64];

  const Dom& D = doms[t.x];
  if (k % D.N_phi || k % D.N_T) return;
  const int nx = D.nx, ny = D.ny, px = D.px, bcx = D.bc[0], bcy = D.bc[1];
  const long long pl = D.plane;
  const int x0 = t.y, ya = t.z, yb = t.w;
  const int w = min(YOW, nx - x0);
  GLOBAL const R* __restrict__ phi_old = gp<const R>(D.phi[qb(n_phi(D, k - 1))]);
  GLOBAL const R* __restrict__ phi_new = gp<const R>(D.phi[qb(n_phi(D, k))]);
  const bool hasU = D.has_U;
  const unsigned nU = (k - 1) / D.N_phi + (k - 1) / D.N_U;
  GLOBAL const R* __restrict__ Uin = hasU ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL R* __restrict__ Uout = hasU ? gp<R>(D.U[qb(nU + 1)]) : nullptr;
  const unsigned nT = n_T(D, k - 1);
  GLOBAL const R* __restrict__ Tin = gp<const R>(D.T[qb(nT)]);
  GLOBAL R* __restrict__ cout = gp<R>(D.T[qb(nT + 2)]);
  GLOBAL const SR* __restrict__ jin = gp<const SR>(D.jT[par(n_jT(D, k - 1))]);
  GLOBAL S* __restrict__ jout = gp<S>(D.jT[par(n_jT(D, k))]);
  GLOBAL const R* __restrict__ vel = D.has_F ? gp<const R>(D.vel[par(n_F(D, k - 1))]) : nullptr;
  const bool need_phi = D.T_var;
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK);
  const R Uref = kc<R>(D, K_U0);   // the U plane holds U - U0
  const R cJ = kc<R>(D, K_CJ);
  const R cT = kc<R>(D, K_CT);
  const R rcS = kc<R>(D, K_RCS), rcL = kc<R>(D, K_RCL);
  const R dt = kc<R>(D, K_DTT);
  const R hkS = kc<R>(D, K_HKS), hkL = kc<R>(D, K_HKL), hrcS = kc<R>(D, K_HRCS), hrcL = kc<R>(D, K_HRCL);
  const R itau_const = rcp(R(3) * dt * kc<R>(D, K_ALPHAL) + R(0.5));
  const R cref = kc<R>(D, K_T0);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const bool wx = bcx != BC_PER, wy = bcy != BC_PER;

  auto put_phi = [&](const YTsIn<R, S>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int cc = tid + 256 * i;
      if (cc < 4 * YBW) wphi[(r0 + 1 + cc / YBW) & 7][cc % YBW] = in.phi[i];
    }
  };
  // J of rows r0 .. r0 + 3 (phi^{q+1} rows r0 - 1 .. r0 + 4 in LDS), as the
  // marching transfer computes it; the gradient of each cell is kept for
  // the T collision of the same cells (the same stencil on the same rows)
  R gsx[2], gsy[2];
  auto flux = [&](const YTsIn<R, S>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int col, row;
      if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
      int rx = x0 - 1 + col, ry = row;
      bool mx = false, my = false;
      if (rx < 0 && bcx != BC_PER) { rx = 0; mx = true; }
      if (rx >= nx && bcx != BC_PER) { rx = nx - 1; mx = true; }
      if (ry < 0 && bcy != BC_PER) { ry = 0; my = true; }
      if (ry >= ny && bcy != BC_PER) { ry = ny - 1; my = true; }
      const int bcol = rx - (x0 - 2);   // window column of the (boundary) node
      R gxv, gyv;
      iso_grad_rows(wphi[(ry - 1) & 7], wphi[ry & 7], wphi[(ry + 1) & 7], bcol, gxv, gyv);
      gsx[i] = gxv;   // at a collision cell (inside the domain) the T collision's grad phi*
      gsy[i] = gyv;
      const R gg = gxv * gxv + gyv * gyv;
      R Jx = R(0), Jy = R(0);
      if (gg >= R(GRAD_EPS2)) {
        const R ig = rsq(gg);
        const R a = cJ * (R(1) + omk * (in.U[i] + Uref)) * (wphi[ry & 7][bcol] - in.po[i]) * ig;
        Jx = -a * gxv;
        Jy = -a * gyv;
      }
      wJx[row & 7][col] = mx ? -Jx : Jx;
      wJy[row & 7][col] = my ? -Jy : Jy;
    }
  };
  // T* and the T collision at the collision cells of rows r0 .. r0 + 3, as
  // the transfer and the marching transport compute them
  auto collide = [&](const YTsIn<R, S>& in, int r0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int col, row;
      if (!ym_cell(i, tx, ty, tid, w, r0, col, row)) continue;
      if (resolve(x0 - 1 + col, nx, bcx) < 0 || resolve(row, ny, bcy) < 0) continue;   // beyond a wall
      const R* r0p = wphi[row & 7];
      const R pn = r0p[col + 1];
      const R dphi = pn - in.po[i];
      const R rc = (R(1) + pn) * R(0.5) * rcS + (R(1) - pn) * R(0.5) * rcL;
      const R dT = cT * dphi * rcp(R(2) * rc);
      const R chi = in.T[i] + dT;
      const R ca = chi + cref;   // the plane holds T - T0
      const R uxv = vel ? in.u[i][0] : R(0), uyv = vel ? in.u[i][1] : R(0);
      const R jxv = cvt_raw(in.j[i][0], (S*)nullptr), jyv = cvt_raw(in.j[i][1], (S*)nullptr);
      const R jex = ca * uxv * dt, jey = ca * uyv * dt;
      R itau, Qs = R(0);
      if (need_phi) {
        const R phi = r0p[col + 1];
        const R irc = rcp((R(1) + phi) * hrcS + (R(1) - phi) * hrcL);
        const R coeff = ((R(1) + phi) * hkS + (R(1) - phi) * hkL) * irc;          // Eq. (11)
        itau = rcp(R(3) * dt * coeff + R(0.5));
        const R gcx = -R(3) * itau * (jxv - jex), gcy = -R(3) * itau * (jyv - jey);
        R gpx, gpy;
        if (hasU) {   // computed with J (the cell is inside the domain: no clamp)
          gpx = gsx[i];
          gpy = gsy[i];
        } else {
          iso_grad_rows(wphi[(row - 1) & 7], r0p, wphi[(row + 1) & 7], col + 1, gpx, gpy);
        }
        Qs = (hrcS - hrcL) * irc * coeff * (gcx * gpx + gcy * gpy);               // Eq. (12), 1st term
      } else {
        itau = itau_const;
      }
      const R om = R(1) - itau;
      R(*cr)[YCW] = wc[row & 7];
      cr[0][col] = chi;
      cr[1][col] = dt * Qs;
      cr[2][col] = jex + om * (jxv - jex);
      cr[3][col] = jey + om * (jyv - jey);
      if constexpr (Q == 9) {
        cr[4][col] = jex;
        cr[5][col] = jey;
      }
    }
  };

  R amax = R(0);
  YTsIn<R, S> in0;
  YTrOwn<R> own;
  // own sites of rows ya .. ya + 3; phi^{q+1} rows ya - 6 .. ya + 1, J and
  // the collisions of rows ya - 3 .. ya
  ym_load_own<R>(ny, px, x0, w, ya + ty, tx, hasU, phi_new, phi_old, Uin, nullptr, own);
  {
    YTsIn<R, S> lo, mid;
    ym_load_ts<R, S>(nx, ny, px, bcx, bcy, x0, w, ya - 7, tx, ty, tid, pl, phi_new, phi_old, Uin, Tin, jin, vel, lo,
                     false);
    ym_load_ts<R, S>(nx, ny, px, bcx, bcy, x0, w, ya - 3, tx, ty, tid, pl, phi_new, phi_old, Uin, Tin, jin, vel, mid);
    put_phi(lo, ya - 7);
    put_phi(mid, ya - 3);
    __syncthreads();
    if (hasU) flux(mid, ya - 3);
    collide(mid, ya - 3);
    ym_load_ts<R, S>(nx, ny, px, bcx, bcy, x0, w, ya + 1, tx, ty, tid, pl, phi_new, phi_old, Uin, Tin, jin, vel, in0);
  }
  __syncthreads();

  for (int y = ya; y < yb; y += 4) {
    // in0: inputs of rows y + 1 .. y + 4, phi^{q+1} rows y + 2 .. y + 5;
    // own: the own site of row y + ty
    put_phi(in0, y + 1);
    const YTsIn<R, S> cur = in0;
    const YTrOwn<R> me = own;
    if (y + 4 < yb) {   // prefetch for the next rows
      ym_load_ts<R, S>(nx, ny, px, bcx, bcy, x0, w, y + 5, tx, ty, tid, pl, phi_new, phi_old, Uin, Tin, jin, vel,
                       in0);
      ym_load_own<R>(ny, px, x0, w, y + 4 + ty, tx, hasU, phi_new, phi_old, Uin, nullptr, own);
    }
    __syncthreads();
    if (hasU) flux(cur, y + 1);
    collide(cur, y + 1);
    __syncthreads();
    const int gy = y + ty;
    // walls tested only on iterations whose rows or column touch one (the
    // test is uniform over the block)
    const bool edge = (wx && (x0 == 0 || x0 + w >= nx)) || (wy && (y == 0 || y + 4 >= ny));
    auto stream_rows = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
      if (tx >= 1 && tx <= w && gy < yb) {
        const int gx = x0 + tx - 1, lx = tx;
        const unsigned o = (unsigned)gy * (unsigned)px + (unsigned)gx;
        if (hasU) {   // U* of the transfer
          const R pn = wphi[gy & 7][lx + 1];
          const R dphi = pn - me.po;
          const int rm = (gy - 1) & 7, r0 = gy & 7, rp = (gy + 1) & 7;
          const R div = (wJx[r0][lx + 1] - wJx[r0][lx - 1]) * R(1.0 / 3.0) +
                        (wJx[rp][lx + 1] - wJx[rp][lx - 1] - wJx[rm][lx - 1] + wJx[rm][lx + 1]) * R(1.0 / 12.0) +
                        (wJy[rp][lx] - wJy[rm][lx]) * R(1.0 / 3.0) +
                        (wJy[rp][lx + 1] + wJy[rp][lx - 1] - wJy[rm][lx - 1] - wJy[rm][lx + 1]) * R(1.0 / 12.0);
          const R Us = me.U;
          const R dU = ((R(1) + omk * (Us + Uref)) * dphi - R(2) * div) * rcp(opk - omk * pn);
          amax = fmax(amax, fabs(dU));
          sto(Uout, o, Us + dU);
        }
        // pull streaming (Eq. 25) of T in deviations d_i = f_i - w_i chi(y)
        const R(*co)[YCW] = wc[gy & 7];
        const R cy = co[0][lx], dPo = co[1][lx];
        R dq[Q];
        dq[0] = dPo * R(Lq::w(0));
#pragma unroll
        for (int q = 1; q < Q; ++q) {
          const int ex = Lq::ex(q), ey = Lq::ey(q);
          const bool wall = EDGE && ((wx && ((ex > 0 && gx == 0) || (ex < 0 && gx == nx - 1))) ||
                                     (wy && ((ey > 0 && gy == 0) || (ey < 0 && gy == ny - 1))));
          if (EDGE && D.T_dirlow && ey > 0 && gy == 0) {
            // anti-bounce-back to T0 at the wall y = -1/2 (the plane holds T - T0)
            dq[q] = -(R(2) * cy + dPo) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, co[2][lx], co[3][lx]);
            if constexpr (Q == 9) dq[q] += R(Lq::cJ(q)) * edot2(ex, ey, co[4][lx], co[5][lx]);
          } else if (wall) {
            dq[q] = dPo * R(Lq::w(q)) - R(Lq::cK) * edot2(ex, ey, co[2][lx], co[3][lx]);
            if constexpr (Q == 9) dq[q] -= R(Lq::cJ(q)) * edot2(ex, ey, co[4][lx], co[5][lx]);
          } else {
            const R(*cu)[YCW] = wc[(gy - ey) & 7];
            const int ux = lx - ex;
            dq[q] = (cu[0][ux] - cy + cu[1][ux]) * R(Lq::w(q)) + R(Lq::cK) * edot2(ex, ey, cu[2][ux], cu[3][ux]);
            if constexpr (Q == 9) dq[q] += R(Lq::cJ(q)) * edot2(ex, ey, cu[4][ux], cu[5][ux]);
          }
        }
        R sum = dq[0];
#pragma unroll
        for (int q = 1; q < Q; ++q) sum += dq[q];
        const R chin = cy + sum;
        sto(cout, o, chin);
        R jx = R(0), jy = R(0);
#pragma unroll
        for (int q = 1; q < Q; ++q) {
          if (Lq::ex(q) > 0) jx += dq[q];
          if (Lq::ex(q) < 0) jx -= dq[q];
          if (Lq::ey(q) > 0) jy += dq[q];
          if (Lq::ey(q) < 0) jy -= dq[q];
        }
        sto(jout, o, jx);
        sto(plane(jout, pl), o, jy);
      }
    };
    if (edge) stream_rows(std::true_type{});
    else stream_rows(std::false_type{});
    __syncthreads();
  }
  if (rmax && hasU) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (tx == 0) red[ty] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int wv = 1; wv < NTHR / 64; ++wv) m = fmax(m, red[wv]);
      double2& P = rmax[ym_run(D, x0, ya)];
      P.x = double(m);
      P.y = double(m);
    }
  }
}

// =================================================================== flow
// D2Q9 MRT (Eq. 27-32) with Guo forcing (Eq. 30), then the weighted partial
// bounce-back of Eq. (33) in pull form with f_L = (1 - phi*)/2, inlet
// equilibrium at x = 0 and zero-gradient outflow at x = nx - 1 when the x
// boundary is inlet/outflow.
#define OPP9(q) ((q) == 0 ? 0 : (q) <= 4 ? (((q) + 1) & 3) + 1 : (((q) - 3) & 3) + 5)

template <class R>
__device__ __forceinline__ void flow_eq(R rho, R ux, R uy, R dt, R* feq) {
  // Eq. (28) with u / c = u dt
  const R u2 = (ux * ux + uy * uy) * dt * dt;
  const R w[9] = {R(4.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9),
                  R(1.0 / 36), R(1.0 / 36), R(1.0 / 36), R(1.0 / 36)};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const R eu = edot2(EX9(i), EY9(i), ux, uy) * dt;
    feq[i] = w[i] * rho * (R(1) + R(3) * eu + R(4.5) * eu * eu - R(1.5) * u2);
  }
}

// MRT collision of Eq. (14) for the flow in deviation form: input rho and
// d_i = f_i - w_i rho (sum_i d_i = 0); output dp_i = f_i^+ - w_i rho.
// The moments of w_i rho are rho (1, -2, 1, 0, ..., 0), so the
// non-equilibrium moments m - m^eq (Eq. 29) follow from M d without
// forming the O(1) populations.
template <class R>
__device__ __forceinline__ void flow_collide(R rho, const R* d, R dt, R Fx, R Fy, R s_e, R s_eps, R s_q,
                                            R s_nu, R* dp) {
  const R c = R(1) / dt;
  // M d with the rows of Eq. (16)
  R md[9];
  md[1] = -R(4) * d[0] - d[1] - d[2] - d[3] - d[4] + R(2) * (d[5] + d[6] + d[7] + d[8]);
  md[2] = R(4) * d[0] - R(2) * (d[1] + d[2] + d[3] + d[4]) + d[5] + d[6] + d[7] + d[8];
  md[3] = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
  md[4] = -R(2) * d[1] + R(2) * d[3] + d[5] - d[6] - d[7] + d[8];
  md[5] = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
  md[6] = -R(2) * d[2] + R(2) * d[4] + d[5] + d[6] - d[7] - d[8];
  md[7] = d[1] - d[2] + d[3] - d[4];
  md[8] = d[5] - d[6] + d[7] - d[8];
  // velocity (Eq. 27) and u / c = u dt
  const R irho = rcp(rho);
  const R ux = (c * md[3] + dt * Fx * R(0.5)) * irho;
  const R uy = (c * md[5] + dt * Fy * R(0.5)) * irho;
  const R Ux = ux * dt, Uy = uy * dt, U2 = Ux * Ux + Uy * Uy;
  // m - m^eq (Eq. 29); the conserved rows 0, 3, 5 relax at rate 0
  R neq[9];
  neq[0] = R(0);
  neq[1] = md[1] - R(3) * rho * U2;
  neq[2] = md[2] + R(3) * rho * U2;
  neq[3] = md[3] - rho * Ux;
  neq[4] = md[4] + rho * Ux;
  neq[5] = md[5] - rho * Uy;
  neq[6] = md[6] + rho * Uy;
  neq[7] = md[7] - rho * (Ux * Ux - Uy * Uy);
  neq[8] = md[8] - rho * Ux * Uy;
  // Guo forcing in moment space (Eq. 30) with 1/c = dt
  const R Fu = (Fx * ux + Fy * uy) * dt * dt;
  const R G[9] = {R(0), R(6) * Fu, -R(6) * Fu, Fx * dt, -Fx * dt, Fy * dt, -Fy * dt,
                  R(2) * (Fx * ux - Fy * uy) * dt * dt, (Fy * ux + Fx * uy) * dt * dt};
  const R sr[9] = {R(0), s_e, s_eps, R(0), s_q, R(0), s_q, s_nu, s_nu};
  R dm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i)   // (the conserved rows relax at rate 0: no multiply by zero issued)
    dm[i] = (i == 0 || i == 3 || i == 5) ? G[i] : -sr[i] * neq[i] + (R(1) - R(0.5) * sr[i]) * G[i];
  // f^+ - f = M^-1 dm, M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
  const R a0 = dm[0] * R(1.0 / 9), a1 = dm[1] * R(1.0 / 36), a2 = dm[2] * R(1.0 / 36);
  const R a3 = dm[3] * R(1.0 / 6), a4 = dm[4] * R(1.0 / 12), a5 = dm[5] * R(1.0 / 6), a6 = dm[6] * R(1.0 / 12);
  const R a7 = dm[7] * R(0.25), a8 = dm[8] * R(0.25);
  dp[0] = d[0] + a0 - R(4) * a1 + R(4) * a2;
  dp[1] = d[1] + a0 - a1 - R(2) * a2 + a3 - R(2) * a4 + a7;
  dp[2] = d[2] + a0 - a1 - R(2) * a2 + a5 - R(2) * a6 - a7;
  dp[3] = d[3] + a0 - a1 - R(2) * a2 - a3 + R(2) * a4 + a7;
  dp[4] = d[4] + a0 - a1 - R(2) * a2 - a5 + R(2) * a6 - a7;
  dp[5] = d[5] + a0 + R(2) * a1 + a2 + a3 + a4 + a5 + a6 + a8;
  dp[6] = d[6] + a0 + R(2) * a1 + a2 - a3 - a4 + a5 + a6 - a8;
  dp[7] = d[7] + a0 + R(2) * a1 + a2 - a3 - a4 - a5 - a6 + a8;
  dp[8] = d[8] + a0 + R(2) * a1 + a2 + a3 + a4 - a5 - a6 - a8;
}

// The nine post-collision planes of a tile live in LDS, so a TY-row tile is
// processed in sub-tiles of SUB rows (8 in FP64, 16 in FP32) that reuse it.
template <class R, class S, int TY, int SUB>
__global__ __launch_bounds__(NTHR) void k_flow(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                unsigned k) {
  constexpr int RPT = SUB / BY;
  constexpr int CW = TX + 2, CH = SUB + 2;
  static_assert(TY % SUB == 0, "tile height must be a multiple of the sub-tile height");
  __shared__ R sfl[CH * CW];
  __shared__ R srho[CH * CW];
  __shared__ R spost[9][CH * CW];   // f_i^+ - w_i rho of the cell

  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  if (k % D.N_F) return;
  const int nx = D.nx, ny = D.ny;
  const int px = D.px;
  const long long pl = D.plane;
  const int fbx = D.fbc[0], fby = D.fbc[1];
  GLOBAL const R* __restrict__ rho_in = gp<const R>(D.rho[par(n_F(D, k - 1))]);
  GLOBAL R* __restrict__ rho_out = gp<R>(D.rho[par(n_F(D, k))]);
  GLOBAL const S* __restrict__ s_in = gp<const S>(D.sF[par(n_F(D, k - 1))]);
  GLOBAL S* __restrict__ s_out = gp<S>(D.sF[par(n_F(D, k))]);
  GLOBAL R* __restrict__ vel = gp<R>(D.vel[par(n_F(D, k))]);
  GLOBAL const R* __restrict__ phis = gp<const R>(D.phi[qb(n_phi(D, k))]);
  const R dt = R(D.N_F * D.dt_base);
  const R Fx = R(D.Fx), Fy = R(D.Fy);
  const R snu = R(1.0 / (3.0 * D.N_F * D.dt_base * D.nu + 0.5));
  const R se = R(D.s_e), seps = R(D.s_eps), sq = R(D.s_q);
  const R w[9] = {R(4.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9),
                  R(1.0 / 36), R(1.0 / 36), R(1.0 / 36), R(1.0 / 36)};
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int x0 = t.y;
  const R c = R(1) / dt;
  const int fbxw = fbx == BC_PER ? BC_PER : BC_WALL, fbyw = fby == BC_PER ? BC_PER : BC_WALL;

  for (int y0 = t.z; y0 < t.z + TY && y0 < ny; y0 += SUB) {
    for (int i = tid; i < CW * CH; i += NTHR) {
      const int lx = i % CW, ly = i / CW;
      const int rx = x0 - 1 + lx, ry = y0 - 1 + ly;
      sfl[i] = (R(1) - ldo(phis, (unsigned)(ghost(ry, ny, fbyw) * px + ghost(rx, nx, fbxw)))) * R(0.5);
      const int gx = resolve(rx, nx, fbxw), gy = resolve(ry, ny, fbyw);
      if (gx < 0 || gy < 0) continue;
      const unsigned o = gy * px + gx;
      const R rho = ldo(rho_in, o);
      R d[9];
      R ssum = R(0);
#pragma unroll
      for (int q = 1; q < 9; ++q) {
        d[q] = ldo(plane(s_in, (q - 1) * pl), o);
        ssum += d[q];
      }
      d[0] = -ssum;
      R dp[9];
      flow_collide(rho, d, dt, Fx, Fy, se, seps, sq, snu, dp);
      srho[i] = rho;
#pragma unroll
      for (int q = 0; q < 9; ++q) spost[q][i] = dp[q];
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int ly = ty + r * BY, gx = x0 + tx, gy = y0 + ly;
      if (gx >= nx || gy >= ny || gy >= t.z + TY) continue;
      if (fbx == BC_INOUT && gx == nx - 1 && nx > 1) continue;  // written by the x = nx-2 site
      const int ci = (ly + 1) * CW + tx + 1;
      // deviations d_i = f_i - w_i rho(y) of the new populations
      R dn[9];
      R rho_y;
      if (fbx == BC_INOUT && gx == 0) {
        // inlet: f = f^eq(1, (u_in, 0))
        rho_y = R(1);
        const R u = R(D.u_in) * dt;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const R eu = R(EX9(q)) * u;
          dn[q] = w[q] * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * u * u);
        }
      } else {
        rho_y = srho[ci];
        const R flo = sfl[ci];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const int ex = EX9(q), ey = EY9(q);
          const int sx = gx - ex, sy = gy - ey;
          const bool out = ((sx < 0 || sx >= nx) && fbx != BC_PER) || ((sy < 0 || sy >= ny) && fby != BC_PER);
          const R bounce = spost[OPP9(q)][ci];
          if (q == 0) {
            dn[0] = spost[0][ci];
          } else if (out) {
            dn[q] = bounce;
          } else {
            const int si = ci - ey * CW - ex;
            const R m = R(0.5) * (flo + sfl[si]);
            dn[q] = m * (w[q] * (srho[si] - rho_y) + spost[q][si]) + (R(1) - m) * bounce;   // Eq. (33)
          }
        }
      }
      R drho = R(0), jx = R(0), jy = R(0);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        drho += dn[q];
        if (EX9(q) != 0) jx += R(EX9(q)) * dn[q];
        if (EY9(q) != 0) jy += R(EY9(q)) * dn[q];
      }
      const R rho = rho_y + drho;
      const R irho = rcp(rho);
      const R ux = (c * jx + dt * Fx * R(0.5)) * irho, uy = (c * jy + dt * Fy * R(0.5)) * irho;
      const int ncopy = (fbx == BC_INOUT && gx == nx - 2) ? 2 : 1;
      for (int cpy = 0; cpy < ncopy; ++cpy) {
        const unsigned o = gy * px + gx + cpy;
        sto(rho_out, o, rho);
        sto(vel, o, ux);
        sto(plane(vel, pl), o, uy);
#pragma unroll
        for (int q = 1; q < 9; ++q) sto(plane(s_out, (q - 1) * pl), o, dn[q] - w[q] * drho);
      }
    }
    __syncthreads();
  }
}

// =================================================================== init
// phi = max over seeds of tanh[(R - r)/(sqrt2 W0)] (Section 4.1); U = U0,
// T = T0, rho = 1, u = 0 or u_in (1 - phi)/2 along x; every population at
// equilibrium with v_n = 0 (Eq. 19, 21, 28).  The U and T planes hold the
// shifts U - U0 and T - T0: far from the interface the increments are many
// orders below the initial value, and adding them to U0 or T0 in FP32 would
// round them away (a systematic solute drift).
template <class R, class S>
__global__ void k_init(const Dom* __restrict__ doms, int dom, const double* __restrict__ xi) {
  const Dom& D = doms[dom];
  const long long n = (long long)D.nx * D.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % D.nx), y = (int)(i / D.nx);
  const long long o = (long long)y * D.px + x, pl = D.plane;
  const double s2w = 1.4142135623730951 * D.W0;
  double phi = -1.0;
  if (xi) {   // planar front along y (Eq. 41)
    phi = tanh((D.z_front + xi[x] - y) / s2w);
  } else {
    for (int s = 0; s < D.nseeds; ++s) {
      const double dx = x - D.seed[s][0], dy = y - D.seed[s][1];
      const double v = tanh((D.seed[s][2] - sqrt(dx * dx + dy * dy)) / s2w);
      phi = v > phi ? v : phi;
    }
  }
  const R ph = R(phi);
  for (int b = 0; b < 4; ++b) (gp<R>(D.phi[b]))[o] = ph;
  if (D.gradeq40)   // the initial equilibrium: v_n = 0, A = 1
    for (int b = 0; b < 2; ++b) {
      (gp<R>(D.gq[b]))[o] = R(0);
      (gp<R>(D.gq[b]))[o + pl] = R(0);
      (gp<R>(D.gq[b]))[o + 2 * pl] = R(1);
    }
  for (int q = 0; q < D.qs - 1; ++q) {
    st(gp<S>(D.sphi[0]), o + q * pl, R(0));
    st(gp<S>(D.sphi[1]), o + q * pl, R(0));
  }
  const double ux = (D.has_F && D.u0_liquid) ? D.u_in * (1.0 - double(ph)) * 0.5 : 0.0;
  if (D.has_U) {
    const double dtU = D.N_U * D.dt_base;
    for (int b = 0; b < 4; ++b) (gp<R>(D.U[b]))[o] = R(0);    // U - U0
    for (int b = 0; b < 2; ++b) {
      (gp<R>(D.jU[b]))[o] = R(D.U0 * ux * dtU);   // the U first moment is stored in R
      (gp<R>(D.jU[b]))[o + pl] = R(0);
    }
    (gp<R>(D.PU))[o] = R(0);
  }
  if (D.has_T) {
    const double dtT = D.N_T * D.dt_base;
    for (int b = 0; b < 4; ++b) (gp<R>(D.T[b]))[o] = R(0);    // T - T0
    for (int b = 0; b < 2; ++b) {
      st(gp<S>(D.jT[b]), o, R(D.T0 * ux * dtT));
      st(gp<S>(D.jT[b]), o + pl, R(0));
    }
    (gp<R>(D.PT))[o] = R(0);
  }
  if (D.has_F) {
    const double dtF = D.N_F * D.dt_base;
    R feq[9];
    flow_eq(R(1), R(ux), R(0), R(dtF), feq);
    const R w[9] = {R(4.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9),
                    R(1.0 / 36), R(1.0 / 36), R(1.0 / 36), R(1.0 / 36)};
    for (int b = 0; b < 2; ++b) {
      (gp<R>(D.rho[b]))[o] = R(1);
      for (int q = 1; q < 9; ++q) st(gp<S>(D.sF[b]), o + (q - 1) * pl, feq[q] - w[q]);
    }
    for (int b = 0; b < 2; ++b) {
      (gp<R>(D.vel[b]))[o] = R(ux);
      (gp<R>(D.vel[b]))[o + pl] = R(0);
    }
  }
}

// =================================================================== read / write
// Plane codes: 0 phi, 1 U, 2 T, 3 rho, 4 ux, 5 uy, 8 U - U0, 9 T - T0
// (the stored planes), 10..14 phase f_0..f_4 (10..18 in D2Q9),
// 20/21 jU, 30/31 jT, 40..48 flow f_0..f_8, 50 pending U, 51 pending T,
// 60..63 stored phase planes s_1..s_4, 70..77 stored flow planes s_1..s_8.
template <class R, class S>
__device__ double read_plane(const Dom& D, long long k, int code, long long o) {
  const long long pl = D.plane;
  switch (code) {
    case 0: return double((gp<const R>(D.phi[qb(n_phi(D, k))]))[o]);
    case 1: return double((gp<const R>(D.U[qb(n_U(D, k))]))[o]) + D.U0;
    case 2: return double((gp<const R>(D.T[qb(n_T(D, k))]))[o]) + D.T0;
    case 8: return double((gp<const R>(D.U[qb(n_U(D, k))]))[o]);
    case 9: return double((gp<const R>(D.T[qb(n_T(D, k))]))[o]);
    case 3: return double((gp<const R>(D.rho[par(n_F(D, k))]))[o]);
    case 4: return double((gp<const R>(D.vel[par(n_F(D, k))]))[o]);
    case 5: return double((gp<const R>(D.vel[par(n_F(D, k))]))[o + pl]);
    case 20: case 21: return double((gp<const R>(D.jU[par(n_jU(D, k))]))[o + (code - 20) * pl]);
    case 30: case 31: return double(ld(gp<const S>(D.jT[par(n_jT(D, k))]), o + (code - 30) * pl));
    case 50: return double((gp<const R>(D.PU))[o]);
    case 51: return double((gp<const R>(D.PT))[o]);
    default: break;
  }
  if (code >= 60 && code < 60 + D.qs - 1)
    return double(ld(gp<const S>(D.sphi[par(n_phi(D, k))]), o + (code - 60) * pl));
  if (code >= 70 && code <= 77) return double(ld(gp<const S>(D.sF[par(n_F(D, k))]), o + (code - 70) * pl));
  if (code >= 10 && code < 10 + D.qs) {
    const int b = par(n_phi(D, k));
    GLOBAL const R* ph = gp<const R>(D.phi[qb(n_phi(D, k))]);
    GLOBAL const S* s = gp<const S>(D.sphi[b]);
    const R phi = ph[o];
    const bool q9 = D.qs == 9;
    if (code == 10) {
      R ssum = R(0);
      for (int q = 0; q < D.qs - 1; ++q) ssum += ld(s, o + q * pl);
      return double(phi * R(q9 ? 4.0 / 9.0 : 1.0 / 3.0) - ssum);
    }
    const int q = code - 10;
    return double(phi * R(q9 ? (q <= 4 ? 1.0 / 9.0 : 1.0 / 36.0) : 1.0 / 6.0) + ld(s, o + (q - 1) * pl));
  }
  if (code >= 40 && code <= 48) {
    const int b = par(n_F(D, k));
    const R rho = (gp<const R>(D.rho[b]))[o];
    GLOBAL const S* s = gp<const S>(D.sF[b]);
    const R w[9] = {R(4.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9),
                    R(1.0 / 36), R(1.0 / 36), R(1.0 / 36), R(1.0 / 36)};
    if (code == 40) {
      R ssum = R(0);
      for (int q = 1; q < 9; ++q) ssum += ld(s, o + (q - 1) * pl);
      return double(w[0] * rho - ssum);
    }
    const int q = code - 40;
    return double(w[q] * rho + ld(s, o + (q - 1) * pl));
  }
  return 0.0;
}

template <class R, class S>
__global__ void k_read(const Dom* __restrict__ doms, int dom, long long k, const int* __restrict__ codes,
                       int ncodes, int out_f64, void* __restrict__ out) {
  const Dom& D = doms[dom];
  const long long n = (long long)D.nx * D.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= ncodes) return;
  const int x = (int)(i % D.nx), y = (int)(i / D.nx);
  const double v = read_plane<R, S>(D, k, codes[c], (long long)y * D.px + x);
  if (out_f64)
    ((double*)out)[c * n + i] = v;
  else
    ((float*)out)[c * n + i] = float(v);
}

// Writes take FP64 planes.  Phase populations (codes 10..14, all five
// present) re-encode phi and s; flow populations (40..48) re-encode rho and s.
template <class R, class S>
__global__ void k_write(const Dom* __restrict__ doms, int dom, long long k, const int* __restrict__ codes,
                        int ncodes, const double* __restrict__ src) {
  const Dom& D = doms[dom];
  const long long n = (long long)D.nx * D.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % D.nx), y = (int)(i / D.nx);
  const long long o = (long long)y * D.px + x, pl = D.plane;
  int cphi = -1, cflow = -1;
  for (int c = 0; c < ncodes; ++c) {
    const int code = codes[c];
    const double v = src[c * n + i];
    switch (code) {
      case 0: (gp<R>(D.phi[qb(n_phi(D, k))]))[o] = R(v); break;
      case 1: (gp<R>(D.U[qb(n_U(D, k))]))[o] = R(v - D.U0); break;
      case 2: (gp<R>(D.T[qb(n_T(D, k))]))[o] = R(v - D.T0); break;
      case 8: (gp<R>(D.U[qb(n_U(D, k))]))[o] = R(v); break;
      case 9: (gp<R>(D.T[qb(n_T(D, k))]))[o] = R(v); break;
      case 3: (gp<R>(D.rho[par(n_F(D, k))]))[o] = R(v); break;
      case 4: (gp<R>(D.vel[par(n_F(D, k))]))[o] = R(v); break;
      case 5: (gp<R>(D.vel[par(n_F(D, k))]))[o + pl] = R(v); break;
      case 20: case 21: (gp<R>(D.jU[par(n_jU(D, k))]))[o + (code - 20) * pl] = R(v); break;
      case 30: case 31: st(gp<S>(D.jT[par(n_jT(D, k))]), o + (code - 30) * pl, R(v)); break;
      case 50: (gp<R>(D.PU))[o] = R(v); break;
      case 51: (gp<R>(D.PT))[o] = R(v); break;
      case 60: case 61: case 62: case 63: case 64: case 65: case 66: case 67:
        if (code < 60 + D.qs - 1) st(gp<S>(D.sphi[par(n_phi(D, k))]), o + (code - 60) * pl, R(v));
        break;
      case 70: case 71: case 72: case 73: case 74: case 75: case 76: case 77:
        st(gp<S>(D.sF[par(n_F(D, k))]), o + (code - 70) * pl, R(v));
        break;
      default:
        if (code == 10) cphi = c;
        if (code == 40) cflow = c;
        break;
    }
  }
  if (cphi >= 0) {
    const int b = par(n_phi(D, k));
    const bool q9 = D.qs == 9;
    R f[9];
    R phi = R(0);
    for (int q = 0; q < D.qs; ++q) {
      f[q] = R(src[(cphi + q) * n + i]);
      phi += f[q];
    }
    (gp<R>(D.phi[qb(n_phi(D, k))]))[o] = phi;
    for (int q = 1; q < D.qs; ++q)
      st(gp<S>(D.sphi[b]), o + (q - 1) * pl, f[q] - phi * R(q9 ? (q <= 4 ? 1.0 / 9.0 : 1.0 / 36.0) : 1.0 / 6.0));
  }
  if (cflow >= 0) {
    const int b = par(n_F(D, k));
    const R w[9] = {R(4.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9),
                    R(1.0 / 36), R(1.0 / 36), R(1.0 / 36), R(1.0 / 36)};
    R f[9];
    R rho = R(0);
    for (int q = 0; q < 9; ++q) {
      f[q] = R(src[(cflow + q) * n + i]);
      rho += f[q];
    }
    (gp<R>(D.rho[b]))[o] = rho;
    for (int q = 1; q < 9; ++q) st(gp<S>(D.sF[b]), o + (q - 1) * pl, f[q] - w[q] * rho);
  }
}

// =================================================================== diagnostics
// Per-tile FP64 partial sums (solid fraction, total solute C of Eq. 5,
// enthalpy for constant properties, mass, non-finite count), reduced across
// the wavefront with shuffles and across the block in LDS.
template <class R, int TY>
__global__ __launch_bounds__(NTHR) void k_diag_tiles(const Dom* __restrict__ doms, const int4* __restrict__ tiles,
                                                      long long k, Partial* __restrict__ part) {
  constexpr int RPT = TY / BY;
  __shared__ double red[5][NTHR / 64];
  const int4 t = tiles[blockIdx.x];
  if (t.x < 0) return;
  const Dom& D = doms[t.x];
  const long long px = D.px;
  GLOBAL const R* phi = gp<const R>(D.phi[qb(n_phi(D, k))]);
  GLOBAL const R* U = D.has_U ? gp<const R>(D.U[qb(n_U(D, k))]) : nullptr;
  GLOBAL const R* T = D.has_T ? gp<const R>(D.T[qb(n_T(D, k))]) : nullptr;
  GLOBAL const R* rho = D.has_F ? gp<const R>(D.rho[par(n_F(D, k))]) : nullptr;
  const int tx = threadIdx.x, ty = threadIdx.y;
  double a[5] = {0, 0, 0, 0, 0};
  for (int r = 0; r < RPT; ++r) {
    const int gx = t.y + tx, gy = t.z + ty + r * BY;
    if (gx >= D.nx || gy >= D.ny) continue;
    const long long o = gy * px + gx;
    const double p = double(phi[o]);
    a[0] += (1.0 + p) * 0.5;
    bool bad = !isfinite(p);
    if (U) {
      const double u = double(U[o]) + D.U0;
      a[1] += D.C_inf * ((1.0 + D.kc) - (1.0 - D.kc) * p) * (1.0 + (1.0 - D.kc) * u) * 0.5;
      bad |= !isfinite(u);
    }
    if (T) {
      const double tv = double(T[o]) + D.T0;
      a[2] += tv - D.rho_L * D.L_h * p / (2.0 * D.rcL);
      bad |= !isfinite(tv);
    }
    if (rho) {
      const double rv = double(rho[o]);
      a[3] += rv;
      bad |= !isfinite(rv);
    }
    a[4] += bad ? 1.0 : 0.0;
  }
  for (int j = 0; j < 5; ++j) {
    double v = a[j];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (tx == 0) red[j][ty] = v;
  }
  __syncthreads();
  if (tx == 0 && ty == 0) {
    double s[5];
    for (int j = 0; j < 5; ++j) {
      s[j] = 0.0;
      for (int w = 0; w < NTHR / 64; ++w) s[j] += red[j][w];
    }
    Partial& P = part[t.w];
    P.solid = s[0];
    P.M_C = s[1];
    P.enthalpy = s[2];
    P.mass = s[3];
    P.nonfinite = s[4];
  }
}

// One block per domain: fixed-order reduction of the tile partials (the
// partial slots of a domain are listed in slot[] in spatial order).
// S_phi and J_U come from whichever kernel last wrote them: the per-run
// maxima when the transfer marched (src bit 0: S_phi, and J_U with
// instantaneous coupling) or, with accumulated coupling, when the U
// transport marched (src bit 1: J_U is the largest injected increment);
// the tile partials otherwise.
__global__ void k_diag_final(const Dom* __restrict__ doms, const Partial* __restrict__ part,
                             const int* __restrict__ slot, const int* __restrict__ slot0,
                             const double2* __restrict__ rmax, int src, DiagOut* __restrict__ out) {
  __shared__ double red[7][4];
  const int d = blockIdx.x;
  const int b = slot0[d], e = slot0[d + 1];
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
    const Partial& P = part[slot[i]];
    a[0] += P.solid;
    a[1] += P.M_C;
    a[2] += P.enthalpy;
    a[3] += P.mass;
    a[4] = fmax(a[4], P.S_phi);
    a[5] = fmax(a[5], P.J_U);
    a[6] += P.nonfinite;
  }
  const Dom& D = doms[d];
  const bool s_runs = (src & 1) != 0, j_runs = (src & (D.accum ? 2 : 1)) != 0;
  if (s_runs || j_runs) {
    double ms = 0.0, mj = 0.0;
    for (int i = D.rbase + threadIdx.x; i < D.rbase + D.nruns; i += blockDim.x) {
      ms = fmax(ms, rmax[i].x);
      mj = fmax(mj, rmax[i].y);
    }
    if (s_runs) a[4] = ms;
    if (j_runs) a[5] = mj;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = 0; j < 7; ++j) {
    double v = a[j];
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(v, off, 64);
      v = (j == 4 || j == 5) ? fmax(v, o) : v + o;
    }
    if (lane == 0) red[j][w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[7];
    for (int j = 0; j < 7; ++j) {
      s[j] = red[j][0];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q) s[j] = (j == 4 || j == 5) ? fmax(s[j], red[j][q]) : s[j] + red[j][q];
    }
    DiagOut& O = out[d];
    O.solid = s[0];
    O.M_C = s[1];
    O.enthalpy = s[2];
    O.mass = s[3];
    O.S_phi = s[4];
    O.J_U = s[5];
    O.nonfinite = (long long)s[6];
  }
}

// Tip distance along one crystal axis of one seed: march outwards at unit
// spacing with bilinear sampling (clamped at the edges); the tip is the
// linear interpolation between the last sample with phi >= 0 and the first
// with phi < 0.  One block per (domain, seed, axis).
template <class R>
__device__ double bilin(const R* phi, long long px, int nx, int ny, double x, double y) {
  x = fmin(fmax(x, 0.0), nx - 1.0);
  y = fmin(fmax(y, 0.0), ny - 1.0);
  int ix = (int)floor(x), iy = (int)floor(y);
  ix = ix > nx - 2 ? nx - 2 : ix;
  iy = iy > ny - 2 ? ny - 2 : iy;
  const double tx = x - ix, ty = y - iy;
  const long long o = iy * px + ix;
  return (1 - tx) * (1 - ty) * double(phi[o]) + tx * (1 - ty) * double(phi[o + 1]) +
         (1 - tx) * ty * double(phi[o + px]) + tx * ty * double(phi[o + px + 1]);
}

template <class R>
__global__ void k_tips(const Dom* __restrict__ doms, long long k, DiagOut* __restrict__ out) {
  __shared__ int sm[4];
  const int d = blockIdx.x, s = blockIdx.y, ax = blockIdx.z;
  const Dom& D = doms[d];
  if (s >= D.nseeds) {
    if (threadIdx.x == 0) out[d].tip[s * 4 + ax] = 0.0;
    return;
  }
  GLOBAL const R* phi = gp<const R>(D.phi[qb(n_phi(D, k))]);
  const double ang = atan2(D.sth, D.cth) + ax * 1.5707963267948966;
  const double c = cos(ang), sn = sin(ang);
  const double cx = D.seed[s][0], cy = D.seed[s][1];
  const int rmax = D.nx > D.ny ? D.nx : D.ny;
  int first = rmax + 1;
  for (int r = threadIdx.x; r <= rmax; r += blockDim.x) {
    if (bilin(phi, D.px, D.nx, D.ny, cx + r * c, cy + r * sn) < 0.0) {
      first = r;
      break;
    }
  }
  for (int off = 32; off > 0; off >>= 1) first = min(first, __shfl_down(first, off, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = first;
  __syncthreads();
  if (threadIdx.x == 0) {
    int f = sm[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) f = min(f, sm[w]);
    double tip;
    if (f == 0)
      tip = 0.0;
    else if (f > rmax)
      tip = double(rmax);
    else {
      const double prev = bilin(phi, D.px, D.nx, D.ny, cx + (f - 1) * c, cy + (f - 1) * sn);
      const double cur = bilin(phi, D.px, D.nx, D.ny, cx + f * c, cy + f * sn);
      tip = (f - 1) + prev / (prev - cur);
    }
    out[d].tip[s * 4 + ax] = tip;
  }
}

// =================================================================== 3D
// Directional solidification in 3D (an extension: the paper's runs are 2D).
// Scalars on D3Q7 (w_0 = 1/4, w_i = 1/8, c_s^2 = 1/4, so the factor 3 of
// Eq. (19), (21), (24), (40) becomes 4), flow on D3Q19, isotropic stencils
// with D3Q19 weights, fourfold-cubic anisotropy a_s = 1 - 3 eps +
// 4 eps sum_a n_a^4.  Every field update marches up through z in one pass
// with its collisions held in LDS (below); x is the fastest index, so every
// plane access is coalesced.
//
// D3Q7 order: 0, +x, -x, +y, -y, +z, -z.  D3Q19 order: 0, the six axes as
// above, then (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1),
// (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1); the opposite
// of q >= 1 is q + 1 for odd q and q - 1 for even q.
__host__ __device__ constexpr int e19(int q, int a) {
  constexpr int E[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                            {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  return E[q][a];
}
__host__ __device__ constexpr int opp19(int q) { return q == 0 ? 0 : (q & 1) ? q + 1 : q - 1; }
__host__ __device__ constexpr double w19(int q) { return q == 0 ? 1.0 / 3 : q <= 6 ? 1.0 / 18 : 1.0 / 36; }

struct Site3 {
  int x, y, z;
  unsigned o;        // offset in a plane (pitch px)
  long long lin;     // x + nx (y + ny z), the packed index of read / write
};

// A block of 256 threads covers 64 x 4 sites of one z plane (x fastest, so
// plane accesses are coalesced rows).  Blocks are dispatched round-robin
// over the 8 XCDs (block b on XCD b mod 8); the columns of tiles are dealt
// to the XCDs and the consecutive blocks of one XCD step up in z through
// the same column, so the z neighbours a block reads were written by the
// same XCD just before and are still in its L2.  The grid has
// pad8(ntx nty) nz blocks (Launch3::blocks); padding blocks have no sites.
__device__ __forceinline__ bool site3(const Dom& D, unsigned b, unsigned t, Site3& s) {
  const unsigned ntx = (unsigned)(D.nx + 63) >> 6, nty = (unsigned)(D.ny + 3) >> 2;
  const unsigned r = b >> 3;
  const unsigned col = (b & 7u) + 8u * (r / (unsigned)D.nz);
  if (col >= ntx * nty) return false;
  const int x = (int)(col % ntx) * 64 + (int)(t & 63u);
  const int y = (int)(col / ntx) * 4 + (int)(t >> 6);
  if (x >= D.nx || y >= D.ny) return false;
  s.x = x;
  s.y = y;
  s.z = (int)(r % (unsigned)D.nz);
  s.o = (unsigned)(((long long)s.z * D.ny + s.y) * D.px + s.x);
  s.lin = ((long long)s.z * D.ny + s.y) * D.nx + s.x;
  return true;
}


// D3Q7 phase collision: (dP, K) and A = a_s^2 from phi, its gradient, j
// (the domain's constants in c, evaluated once on the host)
template <class R>
__device__ __forceinline__ void phase_collide3(const PhaseConst<R>& c, R phi, const R* g, const R* j, R Us, R Ts,
                                               R& dP, R* K, R& A) {
  const R dt = c.dt, W2t = c.W2t, eps = c.eps;
  const R gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  R a_s = R(1), N[3] = {R(0), R(0), R(0)};
  if (gg >= R(GRAD_EPS2)) {
    const R ig = rsq(gg);
    const R gn = gg * ig;
    R n[3], s4 = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      n[a] = -g[a] * ig;
      s4 += n[a] * n[a] * n[a] * n[a];
    }
    a_s = R(1) - R(3) * eps + R(4) * eps * s4;
    const R f = R(-16) * eps * a_s * gn;
#pragma unroll
    for (int a = 0; a < 3; ++a) N[a] = f * n[a] * (n[a] * n[a] - s4);
  }
  A = a_s * a_s;
  const R om = R(1) - rcp(R(4) * dt * A * W2t + R(0.5));   // tau_phi with 1/c_s^2 = 4
  const R theta = (Ts - c.theta_off) * c.inv_lhcp;
  const R q = R(1) - phi * phi;
  const R Q = phi * q - c.lam * (c.Mc * Us + theta) * q * q;
  dP = dt * Q * c.inv_tau0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R je = -W2t * N[a] * dt;
    K[a] = je + om * (j[a] - je);
  }
}

// ------------------------------------------------------------ 3D single pass (z-marching)
// One block owns a 64 x 4 column of sites over a run of z planes and walks
// up through it plane by plane.  Per plane it puts the phase field two
// planes ahead into a four-plane LDS window (the tile plus two rings),
// collides the next plane on the tile plus one ring into a three-plane LDS
// window of (dP, K), and streams the current plane from the planes below,
// at and above.  The collisions stay in LDS (the tile's ring of collisions
// is recomputed by each neighbouring block) instead of making a round trip
// through HBM, and the loads for the next plane are issued before the
// current plane is computed.
constexpr int ZTX = 64, ZTY = 4;                  // tile: one site per thread and plane
constexpr int ZRW = ZTX + 2, ZRH = ZTY + 2;       // collision region (ring 1)
constexpr int ZBW = ZTX + 4, ZBH = ZTY + 4;       // phase window (ring 2)
constexpr int ZNR = ZRW * ZRH, ZNB = ZBW * ZBH;

__device__ __forceinline__ int zslot4(int z) { return (z + 8) & 3; }
__device__ __forceinline__ int zslot3(int z) { return (z + 9) % 3; }

// Domain geometry held in registers for the whole march (the descriptor
// would otherwise be re-read after every store, which may alias it).
struct ZGeo {
  int nx, ny, nz, px, bcx, bcy, bcz;
};
__device__ __forceinline__ ZGeo zgeo(const Dom& D) {
  return ZGeo{D.nx, D.ny, D.nz, D.px, D.bc[0], D.bc[1], D.bc[2]};
}
__device__ __forceinline__ unsigned zoff(const ZGeo& G, int x, int y, int z) {
  return ((unsigned)z * (unsigned)G.ny + (unsigned)y) * (unsigned)G.px + (unsigned)x;
}

// Block -> (tile column, run of z planes).  The (run, column) pairs are
// numbered column fastest and dealt to the 8 XCDs in contiguous ranges
// (block b runs on XCD b mod 8), so neighbouring columns at the same height
// share an XCD and its L2.  The grid has 8 ceil(ncol nrun / 8) blocks.
struct ZCol {
  int x0, y0, w, h, za, zb;
};
template <int TY = ZTY>
__device__ __forceinline__ bool zcol(const ZGeo& G, unsigned b, int zrun, ZCol& c) {
  const int ntx = (G.nx + ZTX - 1) / ZTX, nty = (G.ny + TY - 1) / TY;
  const int ncol = ntx * nty, nrun = (G.nz + zrun - 1) / zrun;
  const int per = (ncol * nrun + 7) / 8;
  const int i = (int)(b >> 3), L = (int)(b & 7u) * per + i;
  if (i >= per || L >= ncol * nrun) return false;
  const int col = L % ncol, run = L / ncol;
  c.x0 = (col % ntx) * ZTX;
  c.y0 = (col / ntx) * TY;
  c.w = min(ZTX, G.nx - c.x0);
  c.h = min(TY, G.ny - c.y0);
  c.za = run * zrun;
  c.zb = min(G.nz, c.za + zrun);
  return true;
}

// region cell i of a thread (0: its own site, 1: a ring cell), in region
// coordinates (the tile is 1..w x 1..h)
__device__ __forceinline__ bool zcell(int i, int tid, const ZCol& c, int& lx, int& ly) {
  if (i == 0) {
    lx = (tid & 63) + 1;
    ly = (tid >> 6) + 1;
    return (tid & 63) < c.w && (tid >> 6) < c.h;
  }
  return ring_cell(tid, c.w, c.h, lx, ly);
}

// isotropic gradient with D3Q19 weights, d_a f = sum_q (3 w_q) e_qa f(x + e_q),
// from the window planes z - 1, z, z + 1 around window cell cb
template <class R>
__device__ __forceinline__ void zgrad(const R* p0, const R* p1, const R* p2, int cb, R* g) {
  g[0] = g[1] = g[2] = R(0);
#pragma unroll
  for (int q = 1; q < 19; ++q) {
    const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2);
    const R* p = ez < 0 ? p0 : ez > 0 ? p2 : p1;
    const R v = p[cb + ey * ZBW + ex];
    const R cq = q <= 6 ? R(1.0 / 6.0) : R(1.0 / 12.0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (e19(q, a) != 0) g[a] += R(e19(q, a)) * cq * v;
  }
}

// window cells of a thread: the in-plane offset of the ghosted site (walls
// clamp to the boundary node, periodic axes wrap).  A 64 x TY tile has
// 64 TY threads and a window of ZBW x (TY + 4) cells.
template <int TY>
struct ZWinT {
  static constexpr int NT = 64 * TY, NB = ZBW * (TY + 4), NBL = (NB + NT - 1) / NT;
};
template <int TY = ZTY>
struct ZWinMap {
  unsigned o[ZWinT<TY>::NBL];    // in-plane offset of the ghosted site
};
template <int TY>
__device__ __forceinline__ void zwin_map(const ZGeo& G, const ZCol& c, int tid, ZWinMap<TY>& m) {
  using W = ZWinT<TY>;
#pragma unroll
  for (int i = 0; i < W::NBL; ++i) {
    const int cc = min(tid + W::NT * i, W::NB - 1);
    const int gx = ghost(c.x0 - 2 + cc % ZBW, G.nx, G.bcx), gy = ghost(c.y0 - 2 + cc / ZBW, G.ny, G.bcy);
    m.o[i] = (unsigned)gy * (unsigned)G.px + (unsigned)gx;
  }
}
template <class R, int TY = ZTY>
struct ZWin {
  R v[ZWinT<TY>::NBL];
};
template <class R, int TY>
__device__ __forceinline__ void zload_win(const ZGeo& G, const ZWinMap<TY>& m, int zw, int tid, GLOBAL const R* f,
                                          ZWin<R, TY>& w) {
  using W = ZWinT<TY>;
  const unsigned pz = (unsigned)ghost(zw, G.nz, G.bcz) * (unsigned)G.ny * (unsigned)G.px;
#pragma unroll
  for (int i = 0; i < W::NBL; ++i)
    if (tid + W::NT * i < W::NB) w.v[i] = ldo(f, pz + m.o[i]);
}
template <class R, int TY>
__device__ __forceinline__ void zput_win(R* dst, const ZWin<R, TY>& w, int tid) {
  using W = ZWinT<TY>;
#pragma unroll
  for (int i = 0; i < W::NBL; ++i)
    if (tid + W::NT * i < W::NB) dst[tid + W::NT * i] = w.v[i];
}

// region cells of a thread: region index and in-plane offset (-1: none,
// or beyond a wall)
struct ZRegMap {
  int cr[2];
  unsigned o[2];
};
// (the region row width ZRW is the same at every tile height)
__device__ __forceinline__ void zreg_map(const ZGeo& G, const ZCol& c, int tid, ZRegMap& m) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    int lx, ly;
    m.cr[i] = -1;
    if (!zcell(i, tid, c, lx, ly)) continue;
    const int gx = resolve(c.x0 - 1 + lx, G.nx, G.bcx), gy = resolve(c.y0 - 1 + ly, G.ny, G.bcy);
    if (gx < 0 || gy < 0) continue;
    m.cr[i] = ly * ZRW + lx;
    m.o[i] = (unsigned)gy * (unsigned)G.px + (unsigned)gx;
  }
}
__device__ __forceinline__ int zbox(int cr) { return (cr / ZRW + 1) * ZBW + cr % ZRW + 1; }

// raw loads of the phase collision inputs of a plane's region cells
template <class R, class S>
struct ZPhaseIn {
  typename RawT<S>::type s[2][6];
  R U[2], T[2];
};
template <class R, class S>
__device__ __forceinline__ void zload_phase(const ZGeo& G, const ZRegMap& m, int zc, long long pl,
                                            GLOBAL const typename RawT<S>::type* sp, GLOBAL const R* Up,
                                            GLOBAL const R* Tp, ZPhaseIn<R, S>& in) {
  const int gz = resolve(zc, G.nz, G.bcz);
  if (gz < 0) return;
  const unsigned pz = (unsigned)gz * (unsigned)G.ny * (unsigned)G.px;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (m.cr[i] < 0) continue;
    const unsigned o = pz + m.o[i];
#pragma unroll
    for (int q = 0; q < 6; ++q) in.s[i][q] = *at(plane(sp, q * pl), o);
    if (Up) in.U[i] = ldo(Up, o);
    if (Tp) in.T[i] = ldo(Tp, o);
  }
}

template <class R, class S, int TY>
__global__ __launch_bounds__(64 * TY) void k3z_phase(const Dom* __restrict__ doms, unsigned k, int zrun) {
  using SR = typename RawT<S>::type;
  constexpr int ZNR = ZRW * (TY + 2), ZNB = ZWinT<TY>::NB;   // collision region and window of a 64 x TY tile
  __shared__ R wphi[4][ZNB];
  __shared__ R wcol[3][4][ZNR];   // dP, Kx, Ky, Kz per region cell
  const Dom& D = doms[0];
  const ZGeo G = zgeo(D);
  ZCol c;
  if (!zcol<TY>(G, blockIdx.x, zrun, c) || k % D.N_phi) return;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const long long pl = D.plane;
  const long long kabs = D.koff + (long long)k;   // absolute base step (rounding streams)
  const unsigned np = n_phi(D, k - 1);
  const int ib = par(np), ob = ib ^ 1;
  GLOBAL const R* phi = gp<const R>(D.phi[qb(np)]);
  GLOBAL const SR* sp = gp<const SR>(D.sphi[ib]);
  GLOBAL R* phi_out = gp<R>(D.phi[qb(np + 1)]);
  GLOBAL S* s_out = gp<S>(D.sphi[ob]);
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  GLOBAL const R* Up = D.has_U ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL const R* Tp = D.has_T ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;
  const PhaseConst<R> pc = phase_const<R>(D);
  const R U0 = kc<R>(D, K_U0), T0 = kc<R>(D, K_T0);
  const bool own = tx < c.w && ty < c.h;
  const int gx = c.x0 + tx, gy = c.y0 + ty;
  ZWinMap<TY> wm;
  zwin_map(G, c, tid, wm);
  ZRegMap rm;
  zreg_map(G, c, tid, rm);
  // upstream neighbours of the own site in x and y (false: beyond a wall)
  const bool upx[2] = {resolve(gx - 1, G.nx, G.bcx) >= 0, resolve(gx + 1, G.nx, G.bcx) >= 0};
  const bool upy[2] = {resolve(gy - 1, G.ny, G.bcy) >= 0, resolve(gy + 1, G.ny, G.bcy) >= 0};
  // whether the block's column touches a wall in x or y
  const bool edge_blk = (G.bcx != BC_PER && (c.x0 == 0 || c.x0 + c.w >= G.nx)) ||
                        (G.bcy != BC_PER && (c.y0 == 0 || c.y0 + c.h >= G.ny));

  // collide plane zc on the region from its loaded inputs and the window
  // planes zc - 1, zc, zc + 1; the own site's A and deviations are returned
  auto collide = [&](const ZPhaseIn<R, S>& in, int zc, R& Aown, R* svown) {
    if (resolve(zc, G.nz, G.bcz) < 0) return;   // beyond a wall: never pulled from
    const R* p0 = wphi[zslot4(zc - 1)];
    const R* p1 = wphi[zslot4(zc)];
    const R* p2 = wphi[zslot4(zc + 1)];
    R* out = &wcol[zslot3(zc)][0][0];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (rm.cr[i] < 0) continue;
      const int cr = rm.cr[i], cb = zbox(cr);
      R g[3];
      zgrad(p0, p1, p2, cb, g);
      R sv[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) sv[q] = cvt_raw(in.s[i][q], (S*)nullptr);
      const R j[3] = {sv[0] - sv[1], sv[2] - sv[3], sv[4] - sv[5]};
      const R Us = Up ? in.U[i] + U0 : R(0);
      const R Ts = Tp ? in.T[i] + T0 : pc.theta_off;
      R dP, K[3], A;
      phase_collide3(pc, p1[cb], g, j, Us, Ts, dP, K, A);
      out[cr] = dP;
      out[ZNR + cr] = K[0];
      out[2 * ZNR + cr] = K[1];
      out[3 * ZNR + cr] = K[2];
      if (i == 0) {
        Aown = A;
#pragma unroll
        for (int q = 0; q < 6; ++q) svown[q] = sv[q];
      }
    }
  };

  // prologue: window planes za - 2 .. za + 1, collisions of za - 1 and za
  R Acur = R(1), Anext = R(1), svcur[6], svnext[6];
  ZPhaseIn<R, S> in0, in1;
  {
    ZWin<R, TY> w0, w1, w2, w3;
    zload_win(G, wm, c.za - 2, tid, phi, w0);
    zload_win(G, wm, c.za - 1, tid, phi, w1);
    zload_win(G, wm, c.za, tid, phi, w2);
    zload_win(G, wm, c.za + 1, tid, phi, w3);
    zload_phase(G, rm, c.za - 1, pl, sp, Up, Tp, in0);
    zload_phase(G, rm, c.za, pl, sp, Up, Tp, in1);
    zput_win(wphi[zslot4(c.za - 2)], w0, tid);
    zput_win(wphi[zslot4(c.za - 1)], w1, tid);
    zput_win(wphi[zslot4(c.za)], w2, tid);
    zput_win(wphi[zslot4(c.za + 1)], w3, tid);
  }
  __syncthreads();
  collide(in0, c.za - 1, Anext, svnext);
  collide(in1, c.za, Acur, svcur);
  ZWin<R, TY> wn;
  zload_win(G, wm, c.za + 2, tid, phi, wn);
  zload_phase(G, rm, c.za + 1, pl, sp, Up, Tp, in0);
  __syncthreads();

  // one plane: `in0` holds the inputs of plane z + 1; once the collision
  // has consumed them the loads for plane z + 2 go to the same registers
  // and are in flight during the streaming.  (Ac, svc) are the own site's
  // A and deviations of plane z, (An, svn) receive those of plane z + 1.
  // The loop runs two planes per iteration with the roles swapped, so no
  // register state is copied between planes.
  auto plane_step = [&](int z, R& Ac, R* svc, R& An, R* svn) {
    zput_win(wphi[zslot4(z + 2)], wn, tid);
    if (z + 1 < c.zb) zload_win(G, wm, z + 3, tid, phi, wn);   // window prefetch
    __syncthreads();
    collide(in0, z + 1, An, svn);   // the plane above: its halo for this plane
    if (z + 1 < c.zb) zload_phase(G, rm, z + 2, pl, sp, Up, Tp, in0);
    __syncthreads();
    // the streaming of a plane that touches no wall (uniform over the
    // block) takes every neighbour from the windows
    auto stream_plane = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
      if (own) {
        // anisotropic pull streaming (Eq. 26) in deviations from w_i phi(y)
        const int cr = (ty + 1) * ZRW + tx + 1, cb = (ty + 2) * ZBW + tx + 2;
        const R* c1 = &wcol[zslot3(z)][0][0];
        const R py = wphi[zslot4(z)][cb];
        const R dPy = c1[cr], Ky[3] = {c1[ZNR + cr], c1[2 * ZNR + cr], c1[3 * ZNR + cr]};
        const R A = Ac, iA = rcp(A), oA = R(1) - A;
        const bool upz[2] = {resolve(z - 1, G.nz, G.bcz) >= 0, resolve(z + 1, G.nz, G.bcz) >= 0};
        R s0 = R(0);
#pragma unroll
        for (int q = 0; q < 6; ++q) s0 -= svc[q];
        R dn[7], sum;
        dn[0] = (dPy * R(0.25) - oA * s0) * iA;
        sum = dn[0];
#pragma unroll
        for (int q = 1; q < 7; ++q) {
          const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2);
          const bool up = !EDGE || (ex > 0 ? upx[0] : ex < 0 ? upx[1] : ey > 0 ? upy[0] : ey < 0 ? upy[1] : ez > 0 ? upz[0] : upz[1]);
          R dpost;
          if (up) {
            const R* cu = &wcol[zslot3(z - ez)][0][0];
            const int ur = cr - ey * ZRW - ex;
            const R Ke = edot3(ex, ey, ez, cu[ZNR + ur], cu[2 * ZNR + ur], cu[3 * ZNR + ur]);
            dpost = (wphi[zslot4(z - ez)][cb - ey * ZBW - ex] - py + cu[ur]) * R(0.125) + R(0.5) * Ke;
          } else {
            dpost = dPy * R(0.125) - R(0.5) * edot3(ex, ey, ez, Ky[0], Ky[1], Ky[2]);
          }
          dn[q] = (dpost - oA * svc[q - 1]) * iA;
          sum += dn[q];
        }
        const unsigned o = zoff(G, gx, gy, z);
        sto(phi_out, o, py + sum);
        SRStream rs = sr_stream(o, kabs, 0x243f6a88u);
#pragma unroll
        for (int q = 1; q < 7; ++q) sto_sr(plane(s_out, (q - 1) * pl), o, dn[q] - R(0.125) * sum, rs);
      }
    };
    if (edge_blk || (G.bcz != BC_PER && (z == 0 || z == G.nz - 1))) stream_plane(std::true_type{});
    else stream_plane(std::false_type{});
    __syncthreads();
  };
  for (int z = c.za; z < c.zb; z += 2) {
    plane_step(z, Acur, svcur, Anext, svnext);
    if (z + 1 < c.zb) plane_step(z + 1, Anext, svnext, Acur, svcur);
  }
}

// raw loads of the scalar collision inputs of a plane's region cells
template <class R, class S>
struct ZScalIn {
  R chi[2];
  typename RawT<S>::type j[2][3];
  R u[2][3];
};
template <class R, class S>
__device__ __forceinline__ void zload_scal(const ZGeo& G, const ZRegMap& m, int zc, long long pl, GLOBAL const R* cin,
                                           GLOBAL const typename RawT<S>::type* jin, GLOBAL const R* vel,
                                           ZScalIn<R, S>& in) {
  const int gz = resolve(zc, G.nz, G.bcz);
  if (gz < 0) return;
  const unsigned pz = (unsigned)gz * (unsigned)G.ny * (unsigned)G.px;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (m.cr[i] < 0) continue;
    const unsigned o = pz + m.o[i];
    in.chi[i] = ldo(cin, o);
#pragma unroll
    for (int a = 0; a < 3; ++a) in.j[i][a] = *at(plane(jin, a * pl), o);
    if (vel) {
#pragma unroll
      for (int a = 0; a < 3; ++a) in.u[i][a] = ldo(plane(vel, a * pl), o);
    }
  }
}

// scalar transport (U: FIELD 0, T: FIELD 1) in one pass: collision to
// (dP, K) on the region of the plane above, pull streaming (Eq. 25) of the
// current plane with bounce-back, or anti-bounce-back to the moving
// profile on the z walls of the pulled T
template <class R, class S, int FIELD, int TY>
__global__ __launch_bounds__(64 * TY) void k3z_scalar(const Dom* __restrict__ doms, unsigned k, int zrun,
                                                  Partial* __restrict__ part) {
  using SR = typename RawT<S>::type;
  constexpr int ZNR = ZRW * (TY + 2), ZNB = ZWinT<TY>::NB;   // collision region and window of a 64 x TY tile
  __shared__ R wphi[4][ZNB];
  // collisions of the planes z and z + 1 (slot z & 1): the streaming of
  // plane z pulls its in-plane neighbours from them; its pulls along z come
  // from the own column's values of planes z - 1 and z + 1, which this
  // thread keeps in registers
  __shared__ R wchi[2][ZNR];
  __shared__ R wcol[2][4][ZNR];   // dP, Kx, Ky, Kz per region cell
  __shared__ R red[TY];
  const Dom& D = doms[0];
  const ZGeo G = zgeo(D);
  const int N = FIELD == 0 ? D.N_U : D.N_T;
  ZCol c;
  if (!zcol<TY>(G, blockIdx.x, zrun, c) || k % N) return;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const long long pl = D.plane;
  const long long kabs = D.koff + (long long)k;   // absolute base step (rounding streams)
  GLOBAL const R* cin;
  GLOBAL R* cout;
  GLOBAL const SR* jin;
  GLOBAL S* jout;
  GLOBAL R* pend;
  if (FIELD == 0) {
    const unsigned nU = (D.accum ? 0u : k / D.N_phi) + (k - 1) / D.N_U;
    cin = gp<const R>(D.U[qb(nU)]);
    cout = gp<R>(D.U[qb(nU + 1)]);
    jin = gp<const SR>(D.jU[par(n_jU(D, k - 1))]);
    jout = gp<S>(D.jU[par(n_jU(D, k))]);
    pend = gp<R>(D.PU);
  } else {
    cin = gp<const R>(D.T[qb(n_Ttr(D, k) + (k - 1) / D.N_T)]);
    cout = gp<R>(D.T[qb(n_Ttr(D, k) + k / D.N_T)]);
    jin = gp<const SR>(D.jT[par(n_jT(D, k - 1))]);
    jout = gp<S>(D.jT[par(n_jT(D, k))]);
    pend = gp<R>(D.PT);
  }
  GLOBAL const R* phis = gp<const R>(D.phi[qb(n_phi(D, k))]);
  GLOBAL const R* vel = D.has_F ? gp<const R>(D.vel[par(n_F(D, k - 1))]) : nullptr;
  const bool var = FIELD == 0 || D.T_var;
  const bool accum = D.accum;
  const R dt = kc<R>(D, FIELD == 0 ? K_DTU : K_DTT);
  const R cref = kc<R>(D, FIELD == 0 ? K_U0 : K_T0);
  const R omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK), DS = kc<R>(D, K_DS), DL = kc<R>(D, K_DL);
  const R hrcS = kc<R>(D, K_HRCS), hrcL = kc<R>(D, K_HRCL), hkS = kc<R>(D, K_HKS), hkL = kc<R>(D, K_HKL);
  const R hdrc = kc<R>(D, K_HDRC);
  const R itau_const = rcp(R(4) * dt * kc<R>(D, K_ALPHAL) + R(0.5));
  const R vpull = FIELD == 1 && D.T_pulled ? R(D.V_pull) : R(0);
  // the walls of the pulled T and of the cold bottom (anti-bounce-back)
  const bool dir = FIELD == 1 && (D.T_pulled || D.T_dirlow), pulled = FIELD == 1 && D.T_pulled;
  const R tmid = R((double(k + D.koff) - 0.5 * N) * D.dt_base);
  const R Tw_lo = pulled ? R(D.T_grad) * (R(-0.5) - R(D.z_front) - R(D.V_pull) * tmid) : R(0);   // T_w - T0
  const R Tw_hi = pulled ? R(D.T_grad) * (R(G.nz - 0.5) - R(D.z_front) - R(D.V_pull) * tmid) : R(0);
  const bool own = tx < c.w && ty < c.h;
  const int gx = c.x0 + tx, gy = c.y0 + ty;
  ZWinMap<TY> wm;
  zwin_map(G, c, tid, wm);
  ZRegMap rm;
  zreg_map(G, c, tid, rm);
  const bool upx[2] = {resolve(gx - 1, G.nx, G.bcx) >= 0, resolve(gx + 1, G.nx, G.bcx) >= 0};
  const bool upy[2] = {resolve(gy - 1, G.ny, G.bcy) >= 0, resolve(gy + 1, G.ny, G.bcy) >= 0};
  // whether the block's column touches a wall in x or y
  const bool edge_blk = (G.bcx != BC_PER && (c.x0 == 0 || c.x0 + c.w >= G.nx)) ||
                        (G.bcy != BC_PER && (c.y0 == 0 || c.y0 + c.h >= G.ny));

  // the own column's (chi - chi_ref, dt Q, K_z) of a plane
  struct OwnZ {
    R chi, dP, Kz;
  };
  auto collide = [&](const ZScalIn<R, S>& in, int zc, OwnZ& ownz) {
    if (resolve(zc, G.nz, G.bcz) < 0) return;   // beyond a wall: never pulled from
    const R* p0 = wphi[zslot4(zc - 1)];
    const R* p1 = wphi[zslot4(zc)];
    const R* p2 = wphi[zslot4(zc + 1)];
    R* out = &wcol[zc & 1][0][0];
    R* cw = wchi[zc & 1];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (rm.cr[i] < 0) continue;
      const int cr = rm.cr[i];
      const R chi = in.chi[i] + cref;   // the plane holds chi - chi_ref
      R u[3] = {R(0), R(0), R(0)};
      if (vel) {
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = in.u[i][a];
      }
      if (FIELD == 1 && pulled) u[2] += vpull;
      R j[3], je[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        j[a] = cvt_raw(in.j[i][a], (S*)nullptr);
        je[a] = chi * u[a] * dt;
      }
      R itau, Q = R(0);
      if (var) {
        const int cb = zbox(cr);
        const R phi = p1[cb];
        R g[3];
        zgrad(p0, p1, p2, cb, g);
        R coeff, pre;
        if (FIELD == 0) {
          const R ikf = rcp(opk - omk * phi);
          coeff = ((R(1) + phi) * DS + (R(1) - phi) * DL) * ikf;            // Eq. (7)
          pre = -omk * coeff * ikf;                                          // Eq. (8), 1st term
        } else {
          const R irc = rcp((R(1) + phi) * hrcS + (R(1) - phi) * hrcL);
          coeff = ((R(1) + phi) * hkS + (R(1) - phi) * hkL) * irc;          // Eq. (11)
          pre = hdrc * irc * coeff;                                          // Eq. (12), 1st term
        }
        itau = rcp(R(4) * dt * coeff + R(0.5));
        R gdot = R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) gdot += -R(4) * itau * (j[a] - je[a]) * g[a];   // Eq. (40), D3Q7
        Q = pre * gdot;
      } else {
        itau = itau_const;
      }
      const R om = R(1) - itau;
      R K[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) K[a] = je[a] + om * (j[a] - je[a]);
      cw[cr] = in.chi[i];
      out[cr] = dt * Q;
#pragma unroll
      for (int a = 0; a < 3; ++a) out[(a + 1) * ZNR + cr] = K[a];
      if (i == 0) ownz = OwnZ{in.chi[i], dt * Q, K[2]};
    }
  };

  R amax = R(0);
  ZScalIn<R, S> in0, in1;
  {
    ZWin<R, TY> w0, w1, w2, w3;
    if (var) {
      zload_win(G, wm, c.za - 2, tid, phis, w0);
      zload_win(G, wm, c.za - 1, tid, phis, w1);
      zload_win(G, wm, c.za, tid, phis, w2);
      zload_win(G, wm, c.za + 1, tid, phis, w3);
    }
    zload_scal(G, rm, c.za - 1, pl, cin, jin, vel, in0);
    zload_scal(G, rm, c.za, pl, cin, jin, vel, in1);
    if (var) {
      zput_win(wphi[zslot4(c.za - 2)], w0, tid);
      zput_win(wphi[zslot4(c.za - 1)], w1, tid);
      zput_win(wphi[zslot4(c.za)], w2, tid);
      zput_win(wphi[zslot4(c.za + 1)], w3, tid);
    }
  }
  __syncthreads();
  // own column at z - 1 and z + 1 (that of z is read back from the
  // window by the streaming, which then keeps it as the next plane's z - 1)
  OwnZ zlo{}, zhi{};
  collide(in0, c.za - 1, zlo);
  collide(in1, c.za, zhi);
  ZWin<R, TY> wn;
  if (var) zload_win(G, wm, c.za + 2, tid, phis, wn);
  zload_scal(G, rm, c.za + 1, pl, cin, jin, vel, in0);
  __syncthreads();

  for (int z = c.za; z < c.zb; ++z) {
    if (var) zput_win(wphi[zslot4(z + 2)], wn, tid);
    if (z + 1 < c.zb && var) zload_win(G, wm, z + 3, tid, phis, wn);   // window prefetch
    __syncthreads();
    collide(in0, z + 1, zhi);
    // the next plane's inputs go to the registers the collision consumed,
    // in flight during the streaming
    if (z + 1 < c.zb) zload_scal(G, rm, z + 2, pl, cin, jin, vel, in0);
    __syncthreads();
    // the streaming of a plane that touches no wall (uniform over the
    // block) takes every neighbour from the windows
    auto stream_plane = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
      if (own) {
        const int cr = (ty + 1) * ZRW + tx + 1;
        const R* c1 = &wcol[z & 1][0][0];
        const R cy = wchi[z & 1][cr], dPy = c1[cr];
        const R Ky[3] = {c1[ZNR + cr], c1[2 * ZNR + cr], c1[3 * ZNR + cr]};
        const bool upz[2] = {resolve(z - 1, G.nz, G.bcz) >= 0, resolve(z + 1, G.nz, G.bcz) >= 0};
        R dq[7];
        dq[0] = dPy * R(0.25);
        R chin = dq[0], j[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int q = 1; q < 7; ++q) {
          const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2);
          const bool up = !EDGE || (ex > 0 ? upx[0] : ex < 0 ? upx[1] : ey > 0 ? upy[0] : ey < 0 ? upy[1] : ez > 0 ? upz[0] : upz[1]);
          if (up && ez != 0) {   // from the own column below or above
            const OwnZ& u = ez > 0 ? zlo : zhi;
            const R Ke = edot3(ex, ey, ez, R(0), R(0), u.Kz);
            dq[q] = (u.chi - cy + u.dP) * R(0.125) + R(0.5) * Ke;
          } else if (up) {
            const R* cu = &wcol[z & 1][0][0];
            const int ur = cr - ey * ZRW - ex;
            const R Ke = edot3(ex, ey, ez, cu[ZNR + ur], cu[2 * ZNR + ur], cu[3 * ZNR + ur]);
            dq[q] = (wchi[z & 1][ur] - cy + cu[ur]) * R(0.125) + R(0.5) * Ke;
          } else {
            const R Ke = edot3(ex, ey, ez, Ky[0], Ky[1], Ky[2]);
            if (dir && (ez > 0 || (ez < 0 && pulled))) {
              const R Tw = ez > 0 ? Tw_lo : Tw_hi;
              dq[q] = R(0.125) * (R(2) * Tw - R(2) * cy - dPy) + R(0.5) * Ke;
            } else {
              dq[q] = dPy * R(0.125) - R(0.5) * Ke;
            }
          }
          chin += dq[q];
          if (ex != 0) j[0] += R(ex) * dq[q];
          if (ey != 0) j[1] += R(ey) * dq[q];
          if (ez != 0) j[2] += R(ez) * dq[q];
        }
        chin += cy;
        const unsigned o = zoff(G, gx, gy, z);
        if (accum) {
          const R p = ldo(pend, o);
          chin += p;
          sto(pend, o, R(0));
          amax = fmax(amax, fabs(p));
        }
        sto(cout, o, chin);
        SRStream rs = sr_stream(o, kabs, FIELD == 0 ? 0x85a308d3u : 0x13198a2eu);
#pragma unroll
        for (int a = 0; a < 3; ++a) sto_sr(plane(jout, a * pl), o, j[a], rs);
        zlo = OwnZ{cy, dPy, Ky[2]};   // the next plane's z - 1
      }
    };
    if (edge_blk || (G.bcz != BC_PER && (z == 0 || z == G.nz - 1))) stream_plane(std::true_type{});
    else stream_plane(std::false_type{});
    __syncthreads();
  }
  if (FIELD == 0 && accum && part) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int i = 1; i < TY; ++i) m = fmax(m, red[i]);
      part[blockIdx.x].J_U = double(m);
    }
  }
}

// raw loads of the transfer inputs of a plane's region cells
template <class R>
struct ZTrIn {
  R po[2], U[2], T;
};
template <class R>
__device__ __forceinline__ void zload_tr(const ZGeo& G, const ZRegMap& m, int zc, GLOBAL const R* po,
                                         GLOBAL const R* Uin, GLOBAL const R* Tin, bool own, ZTrIn<R>& in) {
  const int gz = resolve(zc, G.nz, G.bcz);
  if (gz < 0) return;
  const unsigned pz = (unsigned)gz * (unsigned)G.ny * (unsigned)G.px;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (m.cr[i] < 0) continue;
    const unsigned o = pz + m.o[i];
    in.po[i] = ldo(po, o);
    if (Uin) in.U[i] = ldo(Uin, o);
  }
  if (own && Tin) in.T = ldo(Tin, pz + m.o[0]);
}

// phase-step transfer (Eq. 36-39) in one pass: J = W0/(2 sqrt2) [1 + (1-k)
// U*] dphi n^{q+1} on the region of the plane above, then the compact
// divergence (a neighbour beyond a wall is the boundary node, its J
// mirrored with the normal component negated), dU and dT of Eq. (38) and
// the injection (Eq. 39) on the current plane
template <class R, int TY>
__global__ __launch_bounds__(64 * TY) void k3z_transfer(const Dom* __restrict__ doms, unsigned k, int zrun,
                                                    Partial* __restrict__ part) {
  constexpr int ZNR = ZRW * (TY + 2), ZNB = ZWinT<TY>::NB;   // collision region and window of a 64 x TY tile
  __shared__ R wpn[4][ZNB];
  __shared__ R wJ[3][3][ZNR];
  __shared__ R red[TY];
  const Dom& D = doms[0];
  const ZGeo G = zgeo(D);
  ZCol c;
  if (!zcol<TY>(G, blockIdx.x, zrun, c) || k % D.N_phi) return;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  GLOBAL const R* pn = gp<const R>(D.phi[qb(n_phi(D, k))]);
  GLOBAL const R* po = gp<const R>(D.phi[qb(n_phi(D, k - 1))]);
  const bool hasU = D.has_U, hasT = D.has_T && !D.T_pulled, accum = D.accum;
  const unsigned nU = (D.accum ? 0u : (k - 1) / D.N_phi) + (k - 1) / D.N_U;
  GLOBAL const R* Uin = hasU ? gp<const R>(D.U[qb(nU)]) : nullptr;
  GLOBAL R* Uout = hasU ? gp<R>(D.U[qb(nU + 1)]) : nullptr;
  GLOBAL const R* Tin = hasT ? gp<const R>(D.T[qb(n_T(D, k - 1))]) : nullptr;
  GLOBAL R* Tout = hasT ? gp<R>(D.T[qb(n_T(D, k - 1) + 1)]) : nullptr;
  GLOBAL R* PU = gp<R>(D.PU);
  GLOBAL R* PT = gp<R>(D.PT);
  const R cJ = kc<R>(D, K_CJ), omk = kc<R>(D, K_OMK), opk = kc<R>(D, K_OPK), U0 = kc<R>(D, K_U0);
  const R hrcS = kc<R>(D, K_HRCS), hrcL = kc<R>(D, K_HRCL), cT = kc<R>(D, K_CT);
  const bool own = tx < c.w && ty < c.h;
  const int gx = c.x0 + tx, gy = c.y0 + ty;
  ZWinMap<TY> wm;
  zwin_map(G, c, tid, wm);
  ZRegMap rm;
  zreg_map(G, c, tid, rm);
  // mirror flags of the own site's neighbours in x and y (beyond a wall)
  const bool mxl = gx - 1 < 0 && G.bcx != BC_PER, mxh = gx + 1 >= G.nx && G.bcx != BC_PER;
  const bool myl = gy - 1 < 0 && G.bcy != BC_PER, myh = gy + 1 >= G.ny && G.bcy != BC_PER;
  // whether the block's column touches a wall in x or y
  const bool edge_blk = (G.bcx != BC_PER && (c.x0 == 0 || c.x0 + c.w >= G.nx)) ||
                        (G.bcy != BC_PER && (c.y0 == 0 || c.y0 + c.h >= G.ny));

  // J on the region of plane zc from the window planes zc - 1 .. zc + 1
  auto flux = [&](const ZTrIn<R>& in, int zc) {
    if (resolve(zc, G.nz, G.bcz) < 0) return;   // beyond a wall: the boundary node's J is used
    const R* p0 = wpn[zslot4(zc - 1)];
    const R* p1 = wpn[zslot4(zc)];
    const R* p2 = wpn[zslot4(zc + 1)];
    R* out = &wJ[zslot3(zc)][0][0];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (rm.cr[i] < 0) continue;
      const int cr = rm.cr[i], cb = zbox(cr);
      R g[3];
      zgrad(p0, p1, p2, cb, g);
      const R gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
      R J[3] = {R(0), R(0), R(0)};
      if (gg >= R(GRAD_EPS2)) {
        const R a = cJ * (R(1) + omk * (in.U[i] + U0)) * (p1[cb] - in.po[i]) * rsq(gg);
#pragma unroll
        for (int q = 0; q < 3; ++q) J[q] = -a * g[q];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) out[q * ZNR + cr] = J[q];
    }
  };

  R amax = R(0);
  ZTrIn<R> in0, in1;
  if (hasU) {
    ZWin<R, TY> w0, w1, w2, w3;
    zload_win(G, wm, c.za - 2, tid, pn, w0);
    zload_win(G, wm, c.za - 1, tid, pn, w1);
    zload_win(G, wm, c.za, tid, pn, w2);
    zload_win(G, wm, c.za + 1, tid, pn, w3);
    zload_tr(G, rm, c.za - 1, po, Uin, Tin, false, in0);
    zload_tr(G, rm, c.za, po, Uin, Tin, own, in1);
    zput_win(wpn[zslot4(c.za - 2)], w0, tid);
    zput_win(wpn[zslot4(c.za - 1)], w1, tid);
    zput_win(wpn[zslot4(c.za)], w2, tid);
    zput_win(wpn[zslot4(c.za + 1)], w3, tid);
    __syncthreads();
    flux(in0, c.za - 1);
    flux(in1, c.za);
  } else {
    zload_tr(G, rm, c.za, po, Uin, Tin, own, in1);
  }
  ZTrIn<R> cur = in1;   // inputs of the plane being applied (own cell)
  ZWin<R, TY> wn;
  if (hasU) zload_win(G, wm, c.za + 2, tid, pn, wn);
  zload_tr(G, rm, c.za + 1, po, Uin, Tin, own, in0);
  __syncthreads();

  for (int z = c.za; z < c.zb; ++z) {
    if (hasU) zput_win(wpn[zslot4(z + 2)], wn, tid);
    const ZTrIn<R> nxt = in0;   // inputs of the plane above
    if (z + 1 < c.zb) {         // prefetch for the next plane
      if (hasU) zload_win(G, wm, z + 3, tid, pn, wn);
      zload_tr(G, rm, z + 2, po, Uin, Tin, own, in0);
    }
    __syncthreads();
    if (hasU) flux(nxt, z + 1);
    __syncthreads();
    if (own) {
      const unsigned o = zoff(G, gx, gy, z);
      const int cr = (ty + 1) * ZRW + tx + 1, cb = (ty + 2) * ZBW + tx + 2;
      const R p1 = hasU ? wpn[zslot4(z)][cb] : ldo(pn, o);
      const R dphi = p1 - cur.po[0];
      if (hasU) {
        const bool mzl = z - 1 < 0 && G.bcz != BC_PER, mzh = z + 1 >= G.nz && G.bcz != BC_PER;
        // the divergence of a plane that touches no wall (uniform over the
        // block) takes every neighbour unmirrored
        auto divergence = [&](auto edge_c) {
          constexpr bool EDGE = decltype(edge_c)::value;
          R div = R(0);
#pragma unroll
          for (int q = 1; q < 19; ++q) {
            const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2);
            const bool mir[3] = {EDGE && (ex < 0 ? mxl : ex > 0 ? mxh : false),
                                 EDGE && (ey < 0 ? myl : ey > 0 ? myh : false),
                                 EDGE && (ez < 0 ? mzl : ez > 0 ? mzh : false)};
            // a neighbour beyond a wall is the boundary node itself (ghost)
            const int dx = mir[0] ? 0 : ex, dy = mir[1] ? 0 : ey, dz = mir[2] ? 0 : ez;
            const R* Jq = &wJ[zslot3(z + dz)][0][0];
            const int nr = cr + dy * ZRW + dx;
            const R cq = q <= 6 ? R(1.0 / 6.0) : R(1.0 / 12.0);
#pragma unroll
            for (int a = 0; a < 3; ++a)
              if (e19(q, a) != 0) {
                const R v = Jq[a * ZNR + nr];
                div += R(e19(q, a)) * cq * (mir[a] ? -v : v);
              }
          }
          return div;
        };
        const R div = edge_blk || (G.bcz != BC_PER && (z == 0 || z == G.nz - 1)) ? divergence(std::true_type{})
                                                                                  : divergence(std::false_type{});
        const R Us = cur.U[0];   // U - U0
        const R dU = ((R(1) + omk * (Us + U0)) * dphi - R(2) * div) * rcp(opk - omk * p1);
        amax = fmax(amax, fabs(dU));
        if (accum) sto(PU, o, ldo(PU, o) + dU);
        else sto(Uout, o, Us + dU);
      }
      if (hasT) {
        const R rc = (R(1) + p1) * hrcS + (R(1) - p1) * hrcL;
        const R dT = cT * dphi * rcp(R(2) * rc);
        if (accum) sto(PT, o, ldo(PT, o) + dT);
        else sto(Tout, o, cur.T + dT);
      }
    }
    cur = nxt;
    __syncthreads();
  }
  if (part && hasU) {
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = amax;
    __syncthreads();
    if (tid == 0) {
      R m = red[0];
      for (int i = 1; i < TY; ++i) m = fmax(m, red[i]);
      part[blockIdx.x].S_phi = double(m);
      if (!accum) part[blockIdx.x].J_U = double(m);
    }
  }
}

// D3Q19 MRT in projector form.  The rates are constant on the moment
// subspaces (conserved rho, j: 0; energy: s_e; energy squared: s_eps;
// stress: s_nu; every flux and ghost moment: s_q), so
// M^-1 S M x = s_q x - s_q P_c x - (s_q - s_e) P_e x - (s_q - s_eps) P_eps x
//              - (s_q - s_nu) P_nu x
// with P the orthogonal projectors on the spans of the basis rows
// {1, e_x, e_y, e_z}, {19|e|^2 - 30}, {(21|e|^4 - 53|e|^2 + 24)/2} and
// {3e_x^2 - |e|^2, e_y^2 - e_z^2, e_x e_y, e_y e_z, e_x e_z}.
template <class R>
__device__ __forceinline__ void mrt19_op(const R* x, R sq, R se, R seps, R snu, R* y) {
  // (the basis entries are compile-time constants once the loops are
  // unrolled; the zero ones are skipped, see edot2)
  R c0 = R(0), cx = R(0), cy = R(0), cz = R(0), ce = R(0), cp = R(0), cn[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2), e2 = ex * ex + ey * ey + ez * ez;
    const int kn[5] = {3 * ex * ex - e2, ey * ey - ez * ez, ex * ey, ey * ez, ex * ez};
    c0 += x[q];
    if (ex != 0) cx += R(ex) * x[q];
    if (ey != 0) cy += R(ey) * x[q];
    if (ez != 0) cz += R(ez) * x[q];
    ce += R(19 * e2 - 30) * x[q];
    cp += R((21 * e2 * e2 - 53 * e2 + 24) / 2) * x[q];
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (kn[i] != 0) cn[i] += R(kn[i]) * x[q];
  }
  c0 *= R(1.0 / 19);
  cx *= R(0.1);
  cy *= R(0.1);
  cz *= R(0.1);
  ce *= R(1.0 / 2394);
  cp *= R(1.0 / 252);
  cn[0] *= R(1.0 / 36);
  cn[1] *= R(1.0 / 12);
  cn[2] *= R(0.25);
  cn[3] *= R(0.25);
  cn[4] *= R(0.25);
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2), e2 = ex * ex + ey * ey + ez * ez;
    const int kn[5] = {3 * ex * ex - e2, ey * ey - ez * ez, ex * ey, ey * ez, ex * ez};
    const R pc = c0 + edot3(ex, ey, ez, cx, cy, cz);
    const R pe = ce * R(19 * e2 - 30);
    const R pp = cp * R((21 * e2 * e2 - 53 * e2 + 24) / 2);
    R pn = R(0);
    bool nz = false;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (kn[i] != 0) {
        pn = nz ? pn + cn[i] * R(kn[i]) : cn[i] * R(kn[i]);
        nz = true;
      }
    y[q] = sq * x[q] - sq * pc - (sq - se) * pe - (sq - seps) * pp;
    if (nz) y[q] -= (sq - snu) * pn;
  }
}

// D3Q19 MRT collision of one site (Eq. 27-31 in 3D): the post-collision
// deviations p_q = f_q^+ - w_q rho from rho and the stored deviations d
// (d_0 = -sum of the others)
template <class R>
__device__ __forceinline__ void flow_collide3(R rho, R* d, R dt, R c, const R* F, bool forced, R sq, R se, R seps,
                                             R snu, R* p) {
  R j[3] = {R(0), R(0), R(0)};
  d[0] = R(0);
#pragma unroll
  for (int q = 1; q < 19; ++q) {
    d[0] -= d[q];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (e19(q, a) != 0) j[a] += R(e19(q, a)) * d[q];
  }
  const R irho = rcp(rho);
  R u[3], U[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = (c * j[a] + dt * F[a] * R(0.5)) * irho;     // Eq. (27)
    U[a] = u[a] * dt;
  }
  const R U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  R x[19], Fi[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const R eU = edot3(e19(q, 0), e19(q, 1), e19(q, 2), U[0], U[1], U[2]);
    x[q] = d[q] - R(w19(q)) * rho * (R(3) * eU + R(4.5) * eU * eU - R(1.5) * U2);   // f - f^eq
    if (forced) {
      const R eF = edot3(e19(q, 0), e19(q, 1), e19(q, 2), F[0], F[1], F[2]);
      const R uF = (u[0] * F[0] + u[1] * F[1] + u[2] * F[2]) * dt;
      Fi[q] = R(w19(q)) * (R(3) * (eF - uF) + R(9) * eU * eF) * dt;     // Guo, velocity space
    }
  }
  R y[19];
  mrt19_op(x, sq, se, seps, snu, y);
  if (forced) {
    R yf[19];
    mrt19_op(Fi, sq, se, seps, snu, yf);
#pragma unroll
    for (int q = 0; q < 19; ++q) p[q] = d[q] - y[q] + Fi[q] - R(0.5) * yf[q];
  } else {
#pragma unroll
    for (int q = 0; q < 19; ++q) p[q] = d[q] - y[q];
  }
}

// The unforced D3Q19 collision, by pairs of opposite directions (q, q + 1
// for odd q).  With F_b = 0 the non-equilibrium part x = f - f^eq carries no
// mass and no momentum, so the conserved projector of mrt19_op drops out;
// the odd part of x (momentum, heat flux and ghost vectors, every one but
// the conserved momentum relaxing at s_q) relaxes at s_q alone; and the
// even part needs only the energy, energy-squared and five stress moments,
// sums over x_0 and the nine pair sums x_q + x_qbar.  Per pair the
// equilibrium deviations are B + A and B - A with A = 3 w rho (e.U) and
// B = w rho (4.5 (e.U)^2 - 1.5 U^2), so
//   p_q    = (1 - s_q) d_q    + s_q (B + A) + E_pair,
//   p_qbar = (1 - s_q) d_qbar + s_q (B - A) + E_pair,
// with E_pair the even correction of the pair.  The same relaxation as
// flow_collide3 (equal up to rounding); a quarter of its arithmetic.
template <class R>
__device__ __forceinline__ void flow_collide3_pairs(R rho, R* d, R dt, R c, R sq, R se, R seps, R snu, R* p) {
  R es[9], od[9];
  R sum = R(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    es[k] = d[2 * k + 1] + d[2 * k + 2];
    od[k] = d[2 * k + 1] - d[2 * k + 2];
    sum += es[k];
  }
  d[0] = -sum;
  R j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (e19(2 * k + 1, a) != 0) j[a] += R(e19(2 * k + 1, a)) * od[k];
  const R irho = rcp(rho);
  R U[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) U[a] = (c * j[a]) * irho * dt;   // u dt (Eq. 27, F_b = 0)
  const R U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  R A[9], B[9];
  R x0 = d[0] + R(0.5) * rho * U2;   // B_0 = -1.5 w_0 rho U^2
  R ce = R(-30) * x0, cp = R(12) * x0, cn[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int q = 2 * k + 1;
    const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2), e2 = ex * ex + ey * ey + ez * ez;
    const int kn[5] = {3 * ex * ex - e2, ey * ey - ez * ez, ex * ey, ey * ez, ex * ez};
    const R wr = rho * R(w19(q));
    const R eU = edot3(ex, ey, ez, U[0], U[1], U[2]);
    A[k] = R(3) * wr * eU;
    B[k] = wr * (R(4.5) * eU * eU - R(1.5) * U2);
    const R S = es[k] - R(2) * B[k];     // x_q + x_qbar
    ce += R(19 * e2 - 30) * S;
    cp += R((21 * e2 * e2 - 53 * e2 + 24) / 2) * S;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (kn[i] != 0) cn[i] += R(kn[i]) * S;
  }
  ce *= (sq - se) * R(1.0 / 2394);
  cp *= (sq - seps) * R(1.0 / 252);
  const R an = sq - snu;
  cn[0] *= an * R(1.0 / 36);
  cn[1] *= an * R(1.0 / 12);
  cn[2] *= an * R(0.25);
  cn[3] *= an * R(0.25);
  cn[4] *= an * R(0.25);
  const R om = R(1) - sq;
  p[0] = om * d[0] + sq * (R(-0.5) * rho * U2) + (R(-30) * ce + R(12) * cp);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int q = 2 * k + 1;
    const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2), e2 = ex * ex + ey * ey + ez * ez;
    const int kn[5] = {3 * ex * ex - e2, ey * ey - ez * ez, ex * ey, ey * ez, ex * ez};
    R E = R(19 * e2 - 30) * ce + R((21 * e2 * e2 - 53 * e2 + 24) / 2) * cp;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (kn[i] != 0) E += R(kn[i]) * cn[i];
    const R G = sq * B[k] + E, H = sq * A[k];
    p[q] = om * d[q] + (G + H);
    p[q + 1] = om * d[q + 1] + (G - H);
  }
}

// D3Q19 direction groups by z component: the components a plane streams to
// the plane above (ez = +1), within itself (ez = 0, q >= 1) and below
__host__ __device__ constexpr int zgroup(int q) { return e19(q, 2) > 0 ? 0 : e19(q, 2) == 0 ? 1 : 2; }
__host__ __device__ constexpr int zindex(int q) {   // index of q within its group
  int n = 0;
  for (int r = 1; r < q; ++r) n += zgroup(r) == zgroup(q);
  return n;
}

// raw loads of the flow collision inputs of a plane's region cells
template <class R, class S>
struct ZFlowIn {
  R rho[2], phi[2];
  typename RawT<S>::type s[2][18];
};
template <class R, class S>
__device__ __forceinline__ void zload_flow(const ZGeo& G, const ZRegMap& m, int zc, long long pl, GLOBAL const R* rin,
                                           GLOBAL const R* phis, GLOBAL const typename RawT<S>::type* sp,
                                           ZFlowIn<R, S>& in) {
  const int gz = resolve(zc, G.nz, G.bcz);
  if (gz < 0) return;
  const unsigned pz = (unsigned)gz * (unsigned)G.ny * (unsigned)G.px;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (m.cr[i] < 0) continue;
    const unsigned o = pz + m.o[i];
    in.rho[i] = ldo(rin, o);
    in.phi[i] = ldo(phis, o);
#pragma unroll
    for (int q = 0; q < 18; ++q) in.s[i][q] = *at(plane(sp, q * pl), o);
  }
}

// flow in one pass: MRT collision (Eq. 27-32 in 3D) of the plane above on
// the region, then the partial bounce-back pull (Eq. 33) of the current
// plane in deviations from w_i rho(y).  Components streaming up (ez = +1)
// are kept for two planes, in-plane ones for one, downward ones only for
// the plane being streamed; the own site's nineteen post-collision values
// stay in registers for the bounce-back.
template <class R, class S, int FTY>
__global__ __launch_bounds__(64 * FTY) void k3z_flow(const Dom* __restrict__ doms, unsigned k, int zrun) {
  using SR = typename RawT<S>::type;
  constexpr int ZNR = ZRW * (FTY + 2);   // collision region of a 64 x FTY tile
  __shared__ R wup[3][5][ZNR];     // ez = +1 components, planes z - 1 .. z + 1
  __shared__ R win[2][8][ZNR];     // ez = 0 components, planes z, z + 1
  __shared__ R wdn[5][ZNR];        // ez = -1 components of plane z + 1
  __shared__ R wrho[3][ZNR], wfl[3][ZNR];
  const Dom& D = doms[0];
  const ZGeo G{D.nx, D.ny, D.nz, D.px, D.fbc[0], D.fbc[1], D.fbc[2]};
  ZCol c;
  if (!zcol<FTY>(G, blockIdx.x, zrun, c) || k % D.N_F) return;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const long long pl = D.plane;
  const long long kabs = D.koff + (long long)k;   // absolute base step (rounding streams)
  const int ib = par(n_F(D, k - 1)), ob = par(n_F(D, k));
  GLOBAL const R* rin = gp<const R>(D.rho[ib]);
  GLOBAL const SR* sp = gp<const SR>(D.sF[ib]);
  GLOBAL const R* phis = gp<const R>(D.phi[qb(n_phi(D, k))]);
  GLOBAL R* rho_out = gp<R>(D.rho[ob]);
  GLOBAL R* vel = gp<R>(D.vel[ob]);
  GLOBAL S* s_out = gp<S>(D.sF[ob]);
  const R dt = R(D.N_F * D.dt_base), cdt = R(1) / dt;
  const R F[3] = {R(D.Fx), R(D.Fy), R(D.Fz)};
  const bool forced = D.Fx != 0.0 || D.Fy != 0.0 || D.Fz != 0.0;
  const R snu = R(1.0 / (3.0 * D.N_F * D.dt_base * D.nu + 0.5));
  const R sq = R(D.s_q), se = R(D.s_e), seps = R(D.s_eps);
  const bool own = tx < c.w && ty < c.h;
  const int gx = c.x0 + tx, gy = c.y0 + ty;
  ZRegMap rm;
  zreg_map(G, c, tid, rm);
  const bool upx[2] = {resolve(gx - 1, G.nx, G.bcx) >= 0, resolve(gx + 1, G.nx, G.bcx) >= 0};
  const bool upy[2] = {resolve(gy - 1, G.ny, G.bcy) >= 0, resolve(gy + 1, G.ny, G.bcy) >= 0};
  // whether the block's column touches a wall or an open boundary in x or y
  const bool edge_blk = (G.bcx != BC_PER && (c.x0 == 0 || c.x0 + c.w >= G.nx)) ||
                        (G.bcy != BC_PER && (c.y0 == 0 || c.y0 + c.h >= G.ny));

  // collide plane zc on the region; the own site's values are returned
  auto collide = [&](const ZFlowIn<R, S>& in, int zc, R* pown, R& rown, R& flown) {
    if (resolve(zc, G.nz, G.bcz) < 0) return;   // beyond a wall: never pulled from
    const int su = zslot3(zc), si = zc & 1, s3 = zslot3(zc);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (rm.cr[i] < 0) continue;
      const int cr = rm.cr[i];
      R d[19], p[19];
#pragma unroll
      for (int q = 1; q < 19; ++q) d[q] = cvt_raw(in.s[i][q - 1], (S*)nullptr);
      const R rho = in.rho[i];
      if (forced) flow_collide3(rho, d, dt, cdt, F, true, sq, se, seps, snu, p);
      else flow_collide3_pairs(rho, d, dt, cdt, sq, se, seps, snu, p);
      const R fl = (R(1) - in.phi[i]) * R(0.5);
#pragma unroll
      for (int q = 1; q < 19; ++q) {
        if (zgroup(q) == 0) wup[su][zindex(q)][cr] = p[q];
        else if (zgroup(q) == 1) win[si][zindex(q)][cr] = p[q];
        else wdn[zindex(q)][cr] = p[q];
      }
      wrho[s3][cr] = rho;
      wfl[s3][cr] = fl;
      if (i == 0) {
#pragma unroll
        for (int q = 0; q < 19; ++q) pown[q] = p[q];
        rown = rho;
        flown = fl;
      }
    }
  };

  R pcur[19], pnext[19], rcur = R(1), rnext = R(1), fcur = R(0), fnext = R(0);
  ZFlowIn<R, S> in0;
  {
    ZFlowIn<R, S> a, b;
    zload_flow(G, rm, c.za - 1, pl, rin, phis, sp, a);
    zload_flow(G, rm, c.za, pl, rin, phis, sp, b);
    collide(a, c.za - 1, pnext, rnext, fnext);
    __syncthreads();   // the in-plane and downward components of za - 1 are not needed
    collide(b, c.za, pcur, rcur, fcur);
  }
  zload_flow(G, rm, c.za + 1, pl, rin, phis, sp, in0);
  __syncthreads();

  for (int z = c.za; z < c.zb; ++z) {
    const ZFlowIn<R, S> cur = in0;
    if (z + 1 < c.zb) zload_flow(G, rm, z + 2, pl, rin, phis, sp, in0);   // prefetch
    collide(cur, z + 1, pnext, rnext, fnext);
    __syncthreads();
    // the streaming of a plane that touches no wall (uniform over the
    // block) pulls every direction from the windows
    auto stream_plane = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
      if (!own) return;
      const int cr = (ty + 1) * ZRW + tx + 1;
      const bool upz[2] = {resolve(z - 1, G.nz, G.bcz) >= 0, resolve(z + 1, G.nz, G.bcz) >= 0};
      const R ry = rcur, fly = fcur;
      R dn[19], drho = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
      for (int q = 0; q < 19; ++q) {
        const int ex = e19(q, 0), ey = e19(q, 1), ez = e19(q, 2);
        const R bounce = pcur[opp19(q)];
        if (q == 0) {
          dn[0] = pcur[0];
        } else {
          const bool up = !EDGE || ((ex == 0 || upx[ex > 0 ? 0 : 1]) && (ey == 0 || upy[ey > 0 ? 0 : 1]) &&
                                    (ez == 0 || upz[ez > 0 ? 0 : 1]));
          if (up) {
            const int ur = cr - ey * ZRW - ex, s3 = zslot3(z - ez);
            const R pu = zgroup(q) == 0 ? wup[zslot3(z - 1)][zindex(q)][ur]
                                        : zgroup(q) == 1 ? win[z & 1][zindex(q)][ur] : wdn[zindex(q)][ur];
            const R m = R(0.5) * (fly + wfl[s3][ur]);
            dn[q] = m * (R(w19(q)) * (wrho[s3][ur] - ry) + pu) + (R(1) - m) * bounce;
          } else {
            dn[q] = bounce;
          }
        }
        drho += dn[q];
        if (ex != 0) j[0] += R(ex) * dn[q];
        if (ey != 0) j[1] += R(ey) * dn[q];
        if (ez != 0) j[2] += R(ez) * dn[q];
      }
      const R rho = ry + drho, irho = rcp(rho);
      const unsigned o = zoff(G, gx, gy, z);
      sto(rho_out, o, rho);
#pragma unroll
      for (int a = 0; a < 3; ++a) sto(plane(vel, a * pl), o, (cdt * j[a] + dt * F[a] * R(0.5)) * irho);
      SRStream rs = sr_stream(o, kabs, 0x03707344u);
#pragma unroll
      for (int q = 1; q < 19; ++q) sto_sr(plane(s_out, (q - 1) * pl), o, dn[q] - R(w19(q)) * drho, rs);
    };
    if (edge_blk || (G.bcz != BC_PER && (z == 0 || z == G.nz - 1))) stream_plane(std::true_type{});
    else stream_plane(std::false_type{});
#pragma unroll
    for (int q = 0; q < 19; ++q) pcur[q] = pnext[q];
    rcur = rnext;
    fcur = fnext;
    __syncthreads();
  }
}

// planar front along z at z_front + xi(x, y) (random form of Eq. 41),
// U = U0, T = T0 or the pulled profile, flow at rest; equilibrium
// populations with v_n = 0
template <class R, class S>
__global__ void k3_init(const Dom* __restrict__ doms, const double* __restrict__ xi) {
  const Dom& D = doms[0];
  Site3 s;
  if (!site3(D, blockIdx.x, threadIdx.x, s)) return;
  const unsigned pl = (unsigned)D.plane;
  const double off = xi ? xi[(long long)s.y * D.nx + s.x] : 0.0;
  const double phi = tanh((D.z_front + off - s.z) / (1.4142135623730951 * D.W0));
  for (int b = 0; b < 4; ++b) (gp<R>(D.phi[b]))[s.o] = R(phi);
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < 6; ++q) st(gp<S>(D.sphi[b]), s.o + q * pl, R(0));
  if (D.has_U) {
    for (int b = 0; b < 4; ++b) (gp<R>(D.U[b]))[s.o] = R(0);   // U - U0
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 3; ++a) (gp<R>(D.jU[b]))[s.o + a * pl] = R(0);   // stored in R
    (gp<R>(D.PU))[s.o] = R(0);
  }
  if (D.has_T) {
    const double dT0 = D.T_pulled ? D.T_grad * (s.z - D.z_front) : 0.0;   // T - T0
    const double jz = D.T_pulled ? (D.T0 + dT0) * D.V_pull * D.N_T * D.dt_base : 0.0;
    for (int b = 0; b < 4; ++b) (gp<R>(D.T[b]))[s.o] = R(dT0);
    for (int b = 0; b < 2; ++b) {
      st(gp<S>(D.jT[b]), s.o, R(0));
      st(gp<S>(D.jT[b]), s.o + pl, R(0));
      st(gp<S>(D.jT[b]), s.o + 2 * pl, R(jz));
    }
    (gp<R>(D.PT))[s.o] = R(0);
  }
  if (D.has_F) {
    for (int b = 0; b < 2; ++b) {
      (gp<R>(D.rho[b]))[s.o] = R(1);
      for (int q = 0; q < 18; ++q) st(gp<S>(D.sF[b]), s.o + q * pl, R(0));
      for (int a = 0; a < 3; ++a) (gp<R>(D.vel[b]))[s.o + a * pl] = R(0);
    }
  }
}

// 3D plane codes follow the 2D ones: 0 phi, 1 U, 2 T, 3 rho, 4/5/6 u,
// 8 U - U0, 9 T - T0,
// 10..16 phase f_0..f_6, 20..22 jU, 30..32 jT, 40..58 flow f_0..f_18,
// 50/51 are not used in 3D (pending planes are 90/91), 60..65 phase s,
// 70..87 flow s.
template <class R, class S>
__device__ double read_plane3(const Dom& D, long long k, int code, unsigned o) {
  const unsigned pl = (unsigned)D.plane;
  if (code == 0) return double((gp<const R>(D.phi[qb(n_phi(D, k))]))[o]);
  if (code == 1) return double((gp<const R>(D.U[qb(n_U(D, k))]))[o]) + D.U0;
  if (code == 2) return double((gp<const R>(D.T[qb(n_T(D, k))]))[o]) + D.T0;
  if (code == 8) return double((gp<const R>(D.U[qb(n_U(D, k))]))[o]);
  if (code == 9) return double((gp<const R>(D.T[qb(n_T(D, k))]))[o]);
  if (code == 3) return double((gp<const R>(D.rho[par(n_F(D, k))]))[o]);
  if (code >= 4 && code <= 6) return double((gp<const R>(D.vel[par(n_F(D, k))]))[o + (code - 4) * pl]);
  if (code >= 20 && code <= 22) return double((gp<const R>(D.jU[par(n_jU(D, k))]))[o + (code - 20) * pl]);
  if (code >= 30 && code <= 32) return double(ld(gp<const S>(D.jT[par(n_jT(D, k))]), o + (code - 30) * pl));
  if (code == 90) return double((gp<const R>(D.PU))[o]);
  if (code == 91) return double((gp<const R>(D.PT))[o]);
  if (code >= 60 && code <= 65) return double(ld(gp<const S>(D.sphi[par(n_phi(D, k))]), o + (code - 60) * pl));
  if (code >= 70 && code <= 87) return double(ld(gp<const S>(D.sF[par(n_F(D, k))]), o + (code - 70) * pl));
  if (code >= 10 && code <= 16) {
    const int b = par(n_phi(D, k));
    const R phi = (gp<const R>(D.phi[qb(n_phi(D, k))]))[o];
    GLOBAL const S* sp = gp<const S>(D.sphi[b]);
    if (code == 10) {
      R sum = R(0);
      for (int q = 0; q < 6; ++q) sum += ld(sp, o + q * pl);
      return double(phi * R(0.25) - sum);
    }
    return double(phi * R(0.125) + ld(sp, o + (code - 11) * pl));
  }
  if (code >= 40 && code <= 58) {
    const int b = par(n_F(D, k));
    const R rho = (gp<const R>(D.rho[b]))[o];
    GLOBAL const S* sp = gp<const S>(D.sF[b]);
    if (code == 40) {
      R sum = R(0);
      for (int q = 0; q < 18; ++q) sum += ld(sp, o + q * pl);
      return double(R(w19(0)) * rho - sum);
    }
    const int q = code - 40;
    return double(R(w19(q)) * rho + ld(sp, o + (q - 1) * pl));
  }
  return 0.0;
}

template <class R, class S>
__global__ void k3_read(const Dom* __restrict__ doms, long long k, const int* __restrict__ codes, int ncodes,
                        int out_f64, void* __restrict__ out) {
  const Dom& D = doms[0];
  Site3 s;
  const int c = blockIdx.y;
  if (c >= ncodes || !site3(D, blockIdx.x, threadIdx.x, s)) return;
  const long long n = (long long)D.nx * D.ny * D.nz, i = s.lin;
  const double v = read_plane3<R, S>(D, k, codes[c], s.o);
  if (out_f64)
    ((double*)out)[c * n + i] = v;
  else
    ((float*)out)[c * n + i] = float(v);
}

template <class R, class S>
__global__ void k3_write(const Dom* __restrict__ doms, long long k, const int* __restrict__ codes, int ncodes,
                         const double* __restrict__ src) {
  const Dom& D = doms[0];
  Site3 s;
  if (!site3(D, blockIdx.x, threadIdx.x, s)) return;
  const long long n = (long long)D.nx * D.ny * D.nz, i = s.lin;
  const unsigned o = s.o, pl = (unsigned)D.plane;
  int cphi = -1, cflow = -1;
  for (int c = 0; c < ncodes; ++c) {
    const int code = codes[c];
    const double v = src[c * n + i];
    if (code == 0) (gp<R>(D.phi[qb(n_phi(D, k))]))[o] = R(v);
    else if (code == 1) (gp<R>(D.U[qb(n_U(D, k))]))[o] = R(v - D.U0);
    else if (code == 2) (gp<R>(D.T[qb(n_T(D, k))]))[o] = R(v - D.T0);
    else if (code == 8) (gp<R>(D.U[qb(n_U(D, k))]))[o] = R(v);
    else if (code == 9) (gp<R>(D.T[qb(n_T(D, k))]))[o] = R(v);
    else if (code == 3) (gp<R>(D.rho[par(n_F(D, k))]))[o] = R(v);
    else if (code >= 4 && code <= 6) (gp<R>(D.vel[par(n_F(D, k))]))[o + (code - 4) * pl] = R(v);
    else if (code >= 20 && code <= 22) (gp<R>(D.jU[par(n_jU(D, k))]))[o + (code - 20) * pl] = R(v);
    else if (code >= 30 && code <= 32) st(gp<S>(D.jT[par(n_jT(D, k))]), o + (code - 30) * pl, R(v));
    else if (code == 90) (gp<R>(D.PU))[o] = R(v);
    else if (code == 91) (gp<R>(D.PT))[o] = R(v);
    else if (code >= 60 && code <= 65) st(gp<S>(D.sphi[par(n_phi(D, k))]), o + (code - 60) * pl, R(v));
    else if (code >= 70 && code <= 87) st(gp<S>(D.sF[par(n_F(D, k))]), o + (code - 70) * pl, R(v));
    else if (code == 10) cphi = c;
    else if (code == 40) cflow = c;
  }
  if (cphi >= 0) {
    const int b = par(n_phi(D, k));
    R f[7], phi = R(0);
    for (int q = 0; q < 7; ++q) {
      f[q] = R(src[(cphi + q) * n + i]);
      phi += f[q];
    }
    (gp<R>(D.phi[qb(n_phi(D, k))]))[o] = phi;
    for (int q = 1; q < 7; ++q) st(gp<S>(D.sphi[b]), o + (q - 1) * pl, f[q] - phi * R(0.125));
  }
  if (cflow >= 0) {
    const int b = par(n_F(D, k));
    R f[19], rho = R(0);
    for (int q = 0; q < 19; ++q) {
      f[q] = R(src[(cflow + q) * n + i]);
      rho += f[q];
    }
    (gp<R>(D.rho[b]))[o] = rho;
    for (int q = 1; q < 19; ++q) st(gp<S>(D.sF[b]), o + (q - 1) * pl, f[q] - R(w19(q)) * rho);
  }
}

// FP64 partial sums per block of 256 sites (same quantities as in 2D)
template <class R>
__global__ __launch_bounds__(256) void k3_diag(const Dom* __restrict__ doms, long long k, Partial* __restrict__ part) {
  __shared__ double red[5][4];
  const Dom& D = doms[0];
  Site3 s;
  double a[5] = {0, 0, 0, 0, 0};
  if (site3(D, blockIdx.x, threadIdx.x, s)) {
    const double p = double((gp<const R>(D.phi[qb(n_phi(D, k))]))[s.o]);
    a[0] = (1.0 + p) * 0.5;
    bool bad = !isfinite(p);
    if (D.has_U) {
      const double u = double((gp<const R>(D.U[qb(n_U(D, k))]))[s.o]) + D.U0;
      a[1] = D.C_inf * ((1.0 + D.kc) - (1.0 - D.kc) * p) * (1.0 + (1.0 - D.kc) * u) * 0.5;
      bad |= !isfinite(u);
    }
    if (D.has_T) {
      const double t = double((gp<const R>(D.T[qb(n_T(D, k))]))[s.o]) + D.T0;
      a[2] = t - D.rho_L * D.L_h * p / (2.0 * D.rcL);
      bad |= !isfinite(t);
    }
    if (D.has_F) {
      const double r = double((gp<const R>(D.rho[par(n_F(D, k))]))[s.o]);
      a[3] = r;
      bad |= !isfinite(r);
    }
    a[4] = bad ? 1.0 : 0.0;
  }
  for (int jx = 0; jx < 5; ++jx) {
    double v = a[jx];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[jx][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Partial& P = part[blockIdx.x];
    P.solid = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    P.M_C = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    P.enthalpy = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    P.mass = red[3][0] + red[3][1] + red[3][2] + red[3][3];
    P.nonfinite = red[4][0] + red[4][1] + red[4][2] + red[4][3];
  }
}

// front height per column: the first phi < 0 marching up z, linearly
// interpolated; block max and sum into the partials, reduced on the host
template <class R>
__global__ void k3_front(const Dom* __restrict__ doms, long long k, double* __restrict__ out) {
  __shared__ double rm[4], rs[4];
  const Dom& D = doms[0];
  const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
  double h = 0.0;
  bool has = false;
  if (col < (long long)D.nx * D.ny) {
    has = true;
    const int x = (int)(col % D.nx), y = (int)(col / D.nx);
    GLOBAL const R* phi = gp<const R>(D.phi[qb(n_phi(D, k))]);
    double prev = double(phi[(long long)y * D.px + x]);
    h = prev < 0 ? 0.0 : double(D.nz - 1);
    if (prev >= 0)
      for (int z = 1; z < D.nz; ++z) {
        const double cur = double(phi[((long long)z * D.ny + y) * D.px + x]);
        if (cur < 0) {
          h = (z - 1) + prev / (prev - cur);
          break;
        }
        prev = cur;
      }
  }
  double m = has ? h : -1e300, sm = has ? h : 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_down(m, off, 64));
    sm += __shfl_down(sm, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    rm[threadIdx.x >> 6] = m;
    rs[threadIdx.x >> 6] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = fmax(fmax(rm[0], rm[1]), fmax(rm[2], rm[3]));
    out[2 * blockIdx.x + 1] = rs[0] + rs[1] + rs[2] + rs[3];
  }
}

__global__ void k3_set_koff(Dom* __restrict__ doms, long long koff) {
  if (threadIdx.x == 0) doms[0].koff = koff;
}

template <class R, class S>
struct Launch3 {
  static unsigned blocks(const Dom& h) {
    const long long cols = (long long)((h.nx + 63) / 64) * ((h.ny + 3) / 4);
    return (unsigned)((cols + 7) / 8 * 8 * h.nz);
  }
  // z-marching launches of 64 x ty tiles: runs of zrun planes, enough
  // (column, run) pairs for about zblk blocks of 256 threads (zblk / 2 of
  // 512), runs of at least 8 planes
  static int zrun(const Dom& h, int ty, int zblk) {
    const int ncol = ((h.nx + ZTX - 1) / ZTX) * ((h.ny + ty - 1) / ty);
    const int nrun = std::max(1, std::min((zblk * ZTY / ty + ncol - 1) / ncol, (h.nz + 7) / 8));
    return (h.nz + nrun - 1) / nrun;
  }
  static unsigned zblocks(const Dom& h, int ty, int zblk) {
    const long long ncol = (long long)((h.nx + ZTX - 1) / ZTX) * ((h.ny + ty - 1) / ty);
    const int zr = zrun(h, ty, zblk);
    const long long n = ncol * ((h.nz + zr - 1) / zr);
    return (unsigned)((n + 7) / 8 * 8);
  }
  // rows: tile rows (4 or 8); zblk: the block count the z runs aim at
  static void phase(const Dom& h, hipStream_t st, const Dom* d, unsigned k, int rows, int zblk) {
    if (rows == 8) k3z_phase<R, S, 8><<<zblocks(h, 8, zblk), 512, 0, st>>>(d, k, zrun(h, 8, zblk));
    else k3z_phase<R, S, 4><<<zblocks(h, 4, zblk), 256, 0, st>>>(d, k, zrun(h, 4, zblk));
  }
  static void transfer(const Dom& h, hipStream_t st, const Dom* d, unsigned k, Partial* p, int rows, int zblk) {
    if (rows == 8) k3z_transfer<R, 8><<<zblocks(h, 8, zblk), 512, 0, st>>>(d, k, zrun(h, 8, zblk), p);
    else k3z_transfer<R, 4><<<zblocks(h, 4, zblk), 256, 0, st>>>(d, k, zrun(h, 4, zblk), p);
  }
  static void scalar(int field, const Dom& h, hipStream_t st, const Dom* d, unsigned k, Partial* p, int rows,
                     int zblk) {
    // (the U transport stores its first moment in R: its storage type is R)
    if (rows == 8) {
      const unsigned g = zblocks(h, 8, zblk);
      const int zr = zrun(h, 8, zblk);
      if (field == 0) k3z_scalar<R, R, 0, 8><<<g, 512, 0, st>>>(d, k, zr, p);
      else k3z_scalar<R, S, 1, 8><<<g, 512, 0, st>>>(d, k, zr, p);
    } else {
      const unsigned g = zblocks(h, 4, zblk);
      const int zr = zrun(h, 4, zblk);
      if (field == 0) k3z_scalar<R, R, 0, 4><<<g, 256, 0, st>>>(d, k, zr, p);
      else k3z_scalar<R, S, 1, 4><<<g, 256, 0, st>>>(d, k, zr, p);
    }
  }
  // the flow on 64 x 8 tiles (rows = 8, FP32 arithmetic: 512 threads and
  // 111 KB of LDS, one block per CU) recomputes 1.375 wave collisions per
  // site against 1.75 at 64 x 4, and its barriers then stall the whole CU;
  // in FP64 the LDS window (133 KB at 64 x 4) leaves no room for taller
  // tiles.  Both heights give the same bits.
  static void flow(const Dom& h, hipStream_t st, const Dom* d, unsigned k, int rows, int zblk) {
    if constexpr (sizeof(R) == 4) {
      if (rows == 8) {
        k3z_flow<R, S, 8><<<zblocks(h, 8, zblk), 512, 0, st>>>(d, k, zrun(h, 8, zblk));
        return;
      }
    }
    k3z_flow<R, S, 4><<<zblocks(h, 4, zblk), 256, 0, st>>>(d, k, zrun(h, 4, zblk));
  }
  // rows[5], zblk[5]: tile rows and block targets of the phase, transfer,
  // U, T and flow kernels
  static void step(const Dom& h, hipStream_t st, const Dom* d, unsigned k, Partial* p, const int* rows,
                   const int* zblk) {
    if (k % h.N_phi == 0) {
      phase(h, st, d, k, rows[0], zblk[0]);
      transfer(h, st, d, k, p, rows[1], zblk[1]);
    }
    if (h.has_U && k % h.N_U == 0) scalar(0, h, st, d, k, p, rows[2], zblk[2]);
    if (h.has_T && k % h.N_T == 0) scalar(1, h, st, d, k, p, rows[3], zblk[3]);
    if (h.has_F && k % h.N_F == 0) flow(h, st, d, k, rows[4], zblk[4]);
  }
  static void init(const Dom& h, hipStream_t st, const Dom* d, const double* xi) {
    k3_init<R, S><<<blocks(h), 256, 0, st>>>(d, xi);
  }
  static void set_koff(hipStream_t st, Dom* d, long long koff) { k3_set_koff<<<1, 64, 0, st>>>(d, koff); }
  static void diag(const Dom& h, hipStream_t st, const Dom* d, long long k, Partial* p, double* front) {
    k3_diag<R><<<blocks(h), 256, 0, st>>>(d, k, p);
    k3_front<R><<<(unsigned)(((long long)h.nx * h.ny + 255) / 256), 256, 0, st>>>(d, k, front);
  }
  static void read(const Dom& h, hipStream_t st, const Dom* d, long long k, const int* codes, int nc, int f64,
                   void* out) {
    k3_read<R, S><<<dim3(blocks(h), nc), 256, 0, st>>>(d, k, codes, nc, f64, out);
  }
  static void write(const Dom& h, hipStream_t st, const Dom* d, long long k, const int* codes, int nc,
                    const double* src) {
    k3_write<R, S><<<blocks(h), 256, 0, st>>>(d, k, codes, nc, src);
  }
};

template struct Launch3<double, double>;
template struct Launch3<float, float>;
template struct Launch3<float, __half>;
template struct Launch3<float, __hip_bfloat16>;

// =================================================================== 2D marching launches
// The D2Q5 transfer and scalar transports are compiled for eight waves per
// SIMD (at most 64 VGPRs; without spills): on the batched ensemble the
// fused transfer + T transport went from 0.296 to 0.286 ms, the transfer
// from 0.211 to 0.205 ms.  With BF16 storage the fused transfer + T
// transport would spill at 64 and keeps its own count.  The marching
// phase kernel loads the next rows' inputs into the registers its
// collision has just consumed; with that its D2Q5 form also fits eight
// waves (61 VGPRs; the target caps its SGPRs, which alone held it at
// seven).  The same order in the scalar transports, already at eight
// waves, only shortened their prefetch distance (0.286 -> 0.298 ms).
// Every 2D marching kernel body runs once per column run.  Two launch
// forms share it: a static grid (block b takes run b of an XCD-ordered
// list) and a persistent work queue.  The queue form launches as many
// blocks as fit on the chip; the runs are split into eight lists, one per
// XCD, that hold whole domains (assigned to the lists by longest-
// processing-time packing on their site counts, largest domain first), so
// that the halo rows a run re-reads were loaded into the same XCD's L2 by
// its neighbours.  Block b starts on list b mod 8 (the XCD the dispatcher
// places it on), claims QCHUNK runs at a time and, once that list is
// empty, takes the runs left on the other lists in turn.  Every block
// leaves after finding all eight lists empty.  The counters are rewound by
// k_wq_rewind, launched before the kernel on the same stream.
__global__ void k_wq_rewind(WorkQ* __restrict__ q) {
  if (threadIdx.x < 8) q->next[threadIdx.x][0] = 0u;
}

template <class F>
__device__ __forceinline__ void workq_loop(WorkQ* __restrict__ q, const int4* __restrict__ items,
                                           const int* __restrict__ qoff, F&& body) {
  __shared__ int s_item;
  const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
  const int home = (int)(blockIdx.x & 7u);
  for (int v = 0; v < 8; ++v) {
    const int x = (home + v) & 7;
    const int b = qoff[x], n = qoff[x + 1] - b;
    for (;;) {
      if (lead) s_item = (int)atomicAdd(&q->next[x][0], (unsigned)QCHUNK);
      __syncthreads();
      const int i0 = s_item;
      __syncthreads();
      if (i0 >= n) break;
      const int i1 = min(i0 + QCHUNK, n);
      for (int i = i0; i < i1; ++i) {
        const int4 t = items[b + i];
        if (t.x >= 0) body(t);
        __syncthreads();
      }
    }
  }
}

template <class R, class S, int Q>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(Q == 5 && sizeof(R) == 4 ? 8 : 1))) void k_phase_ym(const Dom* __restrict__ doms, const int4* __restrict__ runs,
                                                    unsigned k) {
  const int4 t = runs[blockIdx.x];
  if (t.x >= 0) k_phase_ym_run<R, S, Q>(doms, t, k);
}
template <class R, class S, int Q>
__global__ __launch_bounds__(NTHR) void k_phase_ym_q(const Dom* __restrict__ doms, const int4* __restrict__ items,
                                                      const int* __restrict__ qoff, WorkQ* __restrict__ q,
                                                      unsigned k) {
  workq_loop(q, items, qoff, [&](const int4 t) { k_phase_ym_run<R, S, Q>(doms, t, k); });
}
template <class R>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1))) void k_transfer_ym(const Dom* __restrict__ doms, const int4* __restrict__ runs,
                                                       unsigned k, double2* __restrict__ rmax) {
  const int4 t = runs[blockIdx.x];
  if (t.x >= 0) k_transfer_ym_run<R>(doms, t, k, rmax);
}
template <class R>
__global__ __launch_bounds__(NTHR) void k_transfer_ym_q(const Dom* __restrict__ doms, const int4* __restrict__ items,
                                                         const int* __restrict__ qoff, WorkQ* __restrict__ q,
                                                         unsigned k, double2* __restrict__ rmax) {
  workq_loop(q, items, qoff, [&](const int4 t) { k_transfer_ym_run<R>(doms, t, k, rmax); });
}
template <class R, class S, int FIELD, int Q>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(Q == 5 && sizeof(R) == 4 ? 8 : 1))) void k_scalar_ym(const Dom* __restrict__ doms, const int4* __restrict__ runs,
                                                     unsigned k, double2* __restrict__ rmax) {
  const int4 t = runs[blockIdx.x];
  if (t.x >= 0) k_scalar_ym_run<R, S, FIELD, Q>(doms, t, k, rmax);
}
template <class R, class S, int FIELD, int Q>
__global__ __launch_bounds__(NTHR) void k_scalar_ym_q(const Dom* __restrict__ doms, const int4* __restrict__ items,
                                                       const int* __restrict__ qoff, WorkQ* __restrict__ q,
                                                       unsigned k, double2* __restrict__ rmax) {
  workq_loop(q, items, qoff, [&](const int4 t) { k_scalar_ym_run<R, S, FIELD, Q>(doms, t, k, rmax); });
}
template <class R, class S, int Q>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(Q == 5 && sizeof(R) == 4 && !std::is_same<S, __hip_bfloat16>::value ? 8 : 1))) void k_tr_scalar_ym(const Dom* __restrict__ doms, const int4* __restrict__ runs,
                                                        unsigned k, double2* __restrict__ rmax) {
  const int4 t = runs[blockIdx.x];
  if (t.x >= 0) k_tr_scalar_ym_run<R, S, Q>(doms, t, k, rmax);
}
template <class R, class S, int Q>
__global__ __launch_bounds__(NTHR) void k_tr_scalar_ym_q(const Dom* __restrict__ doms,
                                                          const int4* __restrict__ items,
                                                          const int* __restrict__ qoff, WorkQ* __restrict__ q,
                                                          unsigned k, double2* __restrict__ rmax) {
  workq_loop(q, items, qoff, [&](const int4 t) { k_tr_scalar_ym_run<R, S, Q>(doms, t, k, rmax); });
}

// =================================================================== launchers
template <class R, class S>
struct Launch {
  // TY selects the tile height: 4, 8, 16 or 32 rows
  // Q: scalar lattice, 5 (D2Q5) or 9 (D2Q9)
  static void phase(int TY, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k) {
    const dim3 b(TX, BY);
    if (Q == 9) {
      if (TY == 4) k_phase<R, S, 4, 9><<<g, b, 0, st>>>(d, t, k);
      else if (TY == 8) k_phase<R, S, 8, 9><<<g, b, 0, st>>>(d, t, k);
      else if (TY == 16) k_phase<R, S, 16, 9><<<g, b, 0, st>>>(d, t, k);
      else k_phase<R, S, 32, 9><<<g, b, 0, st>>>(d, t, k);
      return;
    }
    if (TY == 4) k_phase<R, S, 4, 5><<<g, b, 0, st>>>(d, t, k);
    else if (TY == 8) k_phase<R, S, 8, 5><<<g, b, 0, st>>>(d, t, k);
    else if (TY == 16) k_phase<R, S, 16, 5><<<g, b, 0, st>>>(d, t, k);
    else k_phase<R, S, 32, 5><<<g, b, 0, st>>>(d, t, k);
  }
  // transfer of step k - 1 fused into the phase kernel of step k (D2Q5)
  static void dtr_phase(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p) {
    const dim3 b(TX, BY);
    if (TY == 4) k_dtr_phase<R, S, 4><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 8) k_dtr_phase<R, S, 8><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 16) k_dtr_phase<R, S, 16><<<g, b, 0, st>>>(d, t, k, p);
    else k_dtr_phase<R, S, 32><<<g, b, 0, st>>>(d, t, k, p);
  }
  // transfer of step k fused into the U transport of step k (D2Q5)
  static void dtr_scalar(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p) {
    const dim3 b(TX, BY);
    if (TY == 4) k_dtr_scalar<R, R, 4><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 8) k_dtr_scalar<R, R, 8><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 16) k_dtr_scalar<R, R, 16><<<g, b, 0, st>>>(d, t, k, p);
    else k_dtr_scalar<R, R, 32><<<g, b, 0, st>>>(d, t, k, p);
  }
  // y-marching scalar transport over a list of column runs
  static void scalar_ym(int field, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k,
                        double2* rmax) {
    const dim3 b(TX, BY);
    if (field == 0) {
      if (Q == 9) k_scalar_ym<R, R, 0, 9><<<g, b, 0, st>>>(d, runs, k, rmax);
      else k_scalar_ym<R, R, 0, 5><<<g, b, 0, st>>>(d, runs, k, rmax);
    } else {
      if (Q == 9) k_scalar_ym<R, S, 1, 9><<<g, b, 0, st>>>(d, runs, k, rmax);
      else k_scalar_ym<R, S, 1, 5><<<g, b, 0, st>>>(d, runs, k, rmax);
    }
  }
  // y-marching transfer fused into the T transport of the same step
  static void tr_scalar_ym(int Q, dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k,
                           double2* rmax) {
    const dim3 b(TX, BY);
    if (Q == 9) k_tr_scalar_ym<R, S, 9><<<g, b, 0, st>>>(d, runs, k, rmax);
    else k_tr_scalar_ym<R, S, 5><<<g, b, 0, st>>>(d, runs, k, rmax);
  }
  // y-marching transfer over a list of column runs; slot0: partial slots of
  // the tile height TY in use
  static void transfer_ym(dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k, double2* rmax) {
    k_transfer_ym<R><<<g, dim3(TX, BY), 0, st>>>(d, runs, k, rmax);
  }
  // y-marching phase kernel over a list of column runs
  static void phase_ym(int Q, dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k) {
    const dim3 b(TX, BY);
    if (Q == 9) k_phase_ym<R, S, 9><<<g, b, 0, st>>>(d, runs, k);
    else k_phase_ym<R, S, 5><<<g, b, 0, st>>>(d, runs, k);
  }
  // the same kernels through the per-XCD work queues: as many blocks as
  // fit on the chip (the occupancy of each kernel), at most one per run;
  // the counters are rewound first
  template <class K>
  static unsigned fill(K kern, int nruns, WorkQ* q, hipStream_t st) {
    static std::mutex mu;
    static std::unordered_map<const void*, long long> full;
    long long nb;
    {
      std::lock_guard<std::mutex> lock(mu);
      auto it = full.find((const void*)kern);
      if (it == full.end()) {
        int dev = 0, cus = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
          cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, NTHR, 0) != hipSuccess || n < 1) n = 1;
        it = full.emplace((const void*)kern, (long long)n * cus).first;
      }
      nb = it->second;
    }
    k_wq_rewind<<<1, 64, 0, st>>>(q);
    return (unsigned)std::max(1LL, std::min(nb, (long long)nruns));
  }
  static void phase_ymq(int Q, const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k) {
    const dim3 b(TX, BY);
    if (Q == 9) k_phase_ym_q<R, S, 9><<<fill(k_phase_ym_q<R, S, 9>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k);
    else k_phase_ym_q<R, S, 5><<<fill(k_phase_ym_q<R, S, 5>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k);
  }
  static void transfer_ymq(const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k, double2* rmax) {
    k_transfer_ym_q<R><<<fill(k_transfer_ym_q<R>, l.n, q, st), dim3(TX, BY), 0, st>>>(d, l.items, l.qoff, q, k, rmax);
  }
  static void scalar_ymq(int field, int Q, const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k,
                         double2* rmax) {
    const dim3 b(TX, BY);
    if (field == 0) {
      if (Q == 9) k_scalar_ym_q<R, R, 0, 9><<<fill(k_scalar_ym_q<R, R, 0, 9>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k, rmax);
      else k_scalar_ym_q<R, R, 0, 5><<<fill(k_scalar_ym_q<R, R, 0, 5>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k, rmax);
    } else {
      if (Q == 9) k_scalar_ym_q<R, S, 1, 9><<<fill(k_scalar_ym_q<R, S, 1, 9>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k, rmax);
      else k_scalar_ym_q<R, S, 1, 5><<<fill(k_scalar_ym_q<R, S, 1, 5>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k, rmax);
    }
  }
  static void tr_scalar_ymq(int Q, const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k,
                            double2* rmax) {
    const dim3 b(TX, BY);
    if (Q == 9) k_tr_scalar_ym_q<R, S, 9><<<fill(k_tr_scalar_ym_q<R, S, 9>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k, rmax);
    else k_tr_scalar_ym_q<R, S, 5><<<fill(k_tr_scalar_ym_q<R, S, 5>, l.n, q, st), b, 0, st>>>(d, l.items, l.qoff, q, k, rmax);
  }
  // phase + transfer in one kernel: 8-row tiles in FP64 (LDS), 8 or 16 otherwise
  static int phase_tr_rows(int TY) { return sizeof(R) == 8 ? 8 : (TY >= 16 ? 16 : 8); }
  static void phase_tr(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p) {
    const dim3 b(TX, BY);
    if constexpr (sizeof(R) == 8) {
      k_phase_tr<R, S, 8><<<g, b, 0, st>>>(d, t, k, p);
    } else {
      if (TY >= 16) k_phase_tr<R, S, 16><<<g, b, 0, st>>>(d, t, k, p);
      else k_phase_tr<R, S, 8><<<g, b, 0, st>>>(d, t, k, p);
    }
  }
  static void transfer(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p) {
    const dim3 b(TX, BY);
    if (TY == 4) k_transfer<R, 4><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 8) k_transfer<R, 8><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 16) k_transfer<R, 16><<<g, b, 0, st>>>(d, t, k, p);
    else k_transfer<R, 32><<<g, b, 0, st>>>(d, t, k, p);
  }
  // SF: storage type of the field's first moment (R for U, S for T)
  template <int F, class SF>
  static void scalar_f(int TY, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k,
                       Partial* p) {
    const dim3 b(TX, BY);
    if (Q == 9) {
      if (TY == 4) k_scalar<R, SF, 4, F, 9><<<g, b, 0, st>>>(d, t, k, p);
      else if (TY == 8) k_scalar<R, SF, 8, F, 9><<<g, b, 0, st>>>(d, t, k, p);
      else if (TY == 16) k_scalar<R, SF, 16, F, 9><<<g, b, 0, st>>>(d, t, k, p);
      else k_scalar<R, SF, 32, F, 9><<<g, b, 0, st>>>(d, t, k, p);
      return;
    }
    if (TY == 4) k_scalar<R, SF, 4, F, 5><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 8) k_scalar<R, SF, 8, F, 5><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 16) k_scalar<R, SF, 16, F, 5><<<g, b, 0, st>>>(d, t, k, p);
    else k_scalar<R, SF, 32, F, 5><<<g, b, 0, st>>>(d, t, k, p);
  }
  static void scalar(int field, int TY, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k,
                     Partial* p) {
    // the U transport stores its first moment in R (solute conservation is
    // the accuracy target of the reduced-precision formats)
    if (field == 0) scalar_f<0, R>(TY, Q, g, st, d, t, k, p);
    else scalar_f<1, S>(TY, Q, g, st, d, t, k, p);
  }
  static void flow(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k) {
    constexpr int SUB = sizeof(R) == 8 ? 8 : 16;
    const dim3 b(TX, BY);
    if (TY == 4) k_flow<R, S, 4, 4><<<g, b, 0, st>>>(d, t, k);
    else if (TY == 8) k_flow<R, S, 8, 8><<<g, b, 0, st>>>(d, t, k);
    else if (TY == 16) k_flow<R, S, 16, SUB><<<g, b, 0, st>>>(d, t, k);
    else k_flow<R, S, 32, SUB><<<g, b, 0, st>>>(d, t, k);
  }
  static void diag_tiles(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, long long k, Partial* p) {
    const dim3 b(TX, BY);
    if (TY == 4) k_diag_tiles<R, 4><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 8) k_diag_tiles<R, 8><<<g, b, 0, st>>>(d, t, k, p);
    else if (TY == 16) k_diag_tiles<R, 16><<<g, b, 0, st>>>(d, t, k, p);
    else k_diag_tiles<R, 32><<<g, b, 0, st>>>(d, t, k, p);
  }
  static void tips(int ndom, hipStream_t st, const Dom* d, long long k, DiagOut* o) {
    k_tips<R><<<dim3(ndom, MAX_SEEDS, 4), 256, 0, st>>>(d, k, o);
  }
  static void init(hipStream_t st, const Dom* d, int dom, long long n, const double* xi) {
    k_init<R, S><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(d, dom, xi);
  }
  static void read(hipStream_t st, const Dom* d, int dom, long long k, const int* codes, int nc, int f64,
                   void* out, long long n) {
    k_read<R, S><<<dim3((unsigned)((n + 255) / 256), nc), 256, 0, st>>>(d, dom, k, codes, nc, f64, out);
  }
  static void write(hipStream_t st, const Dom* d, int dom, long long k, const int* codes, int nc,
                    const double* src, long long n) {
    k_write<R, S><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(d, dom, k, codes, nc, src);
  }
};

void diag_final(int ndom, hipStream_t st, const Dom* d, const Partial* p, const int* slot, const int* slot0,
                const double2* rmax, int src, DiagOut* o) {
  k_diag_final<<<ndom, 256, 0, st>>>(d, p, slot, slot0, rmax, src, o);
}

// Non-finite screen of the macroscopic planes after base step k (absolute):
// block (x, d) walks rows x, x + gridDim.x, ... (four per block) of domain
// d's phi, U, T and rho planes (their latest buffers); a wavefront that
// meets a NaN or an infinity lowers first[d] to k with an atomic minimum.
// A diverging field reaches phi within a few steps (U and T enter the phase
// source, the flow advects U and T), and these are the planes every kernel
// reads, so the screen stays a plain read of four planes per check.
template <class R>
__global__ __launch_bounds__(256) void k_nonfinite(const Dom* __restrict__ doms, long long k,
                                                   unsigned long long* __restrict__ first) {
  const Dom& D = doms[blockIdx.y];
  GLOBAL const R* pl[4];
  int np = 0;
  pl[np++] = gp<const R>(D.phi[qb(n_phi(D, k))]);
  if (D.has_U) pl[np++] = gp<const R>(D.U[qb(n_U(D, k))]);
  if (D.has_T) pl[np++] = gp<const R>(D.T[qb(n_T(D, k))]);
  if (D.has_F) pl[np++] = gp<const R>(D.rho[par(n_F(D, k))]);
  const long long rows = (long long)D.ny * D.nz;
  bool bad = false;
  for (long long r = (long long)blockIdx.x * 4 + threadIdx.y; r < rows; r += (long long)gridDim.x * 4)
    for (int x = threadIdx.x; x < D.nx; x += 64) {
      const long long o = r * D.px + x;
      for (int p = 0; p < np; ++p) bad |= !isfinite(pl[p][o]);
    }
  if (__ballot(bad) && threadIdx.x == 0) atomicMin(&first[blockIdx.y], (unsigned long long)k);
}

void nonfinite_check(int f64, int ndom, int blocks, hipStream_t st, const Dom* d, long long k,
                     unsigned long long* first) {
  if (f64) k_nonfinite<double><<<dim3(blocks, ndom), dim3(64, 4), 0, st>>>(d, k, first);
  else k_nonfinite<float><<<dim3(blocks, ndom), dim3(64, 4), 0, st>>>(d, k, first);
}

template struct Launch<double, double>;
template struct Launch<float, float>;
template struct Launch<float, __half>;
template struct Launch<float, __hip_bfloat16>;

}  // namespace lbm
