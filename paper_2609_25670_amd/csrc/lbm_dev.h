// Device-side data model shared by the kernels and the host runtime of the
// multirate lattice-Boltzmann library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int TX = 64;        // tile width: one wavefront across x
constexpr int BY = 4;         // thread rows per block (256 threads)
constexpr int NTHR = TX * BY;
constexpr int MAX_SEEDS = 4;
// 2D marching runs: YCOL columns (plus one ring cell each side: one
// wavefront) by YRUN rows (a multiple of every tile height)
constexpr int YCOL = 62, YRUN = 64;
// |grad phi|^2 below which the interface normal is taken as zero (a_s = 1,
// N = 0, no anti-trapping current): gradients of 1e-8 and less are far below
// the interface scale and their direction is not resolved in FP64.
constexpr double GRAD_EPS2 = 1e-16;

enum Bc { BC_PER = 0, BC_WALL = 1, BC_INOUT = 2 };

// Derived per-domain constants of the 2D kernels, evaluated once on the host
// in FP64 (kd) and rounded to FP32 (kf), so no kernel spends FP64 divisions
// or conversions on them.
enum Kc {
  K_DTPHI, K_W2T, K_INVTAU0, K_EPS, K_LAM, K_MC, K_CTH, K_STH, K_INVLHCP, K_THOFF,
  K_OMK, K_OPK, K_CJ, K_CT, K_RCS, K_RCL, K_HRCS, K_HRCL, K_HKS, K_HKL, K_DTU, K_DTT,
  K_DS, K_DL, K_U0, K_T0, K_ALPHAL, K_HDRC, K_DTF, K_N
};

// Per-domain device descriptor.  Pointers address planes of px*ny elements
// (pitch px, x fastest).  R = FP64 when the context stores FP64, else FP32;
// S = the population storage type.
struct Dom {
  int nx, ny, nz, px;           // nz = 1 in 2D
  long long plane;              // elements per plane (px * ny * nz)
  int bc[3];                    // scalar boundaries (x, y, z)
  int fbc[3];                   // flow boundaries (x, y, z)
  int N_phi, N_U, N_T, N_F;
  int has_U, has_T, has_F, accum;
  int T_var;                    // thermal properties vary with phi
  int T_pulled;                 // 3D pulled temperature (no latent heat, moving walls)
  int T_dirlow;                 // low wall of the last axis held at T0 (latent heat kept)
  int dim;
  int tile0;                    // first tile slot of this domain (partials)
  int ntiles;                   // tiles of this domain
  int nseeds;
  double seed[MAX_SEEDS][3];    // x, y, R
  double dt_base, W0, tau0, eps, lam, Mc, kc, cth, sth;
  double D_L, D_S, C_inf;
  double kS, kL, rcS, rcL, rho_L, L_h, T_m, m_L, Cp_L;
  double nu, s_e, s_eps, s_q, u_in, Fx, Fy, Fz;
  double U0, T0;
  double T_grad, V_pull, z_front;
  int u0_liquid;
  int qs;                       // scalar lattice: 5 (D2Q5), 9 (D2Q9) or 7 (D3Q7)
  int rbase, nruns;             // 2D: first index and count of the domain's marching runs
  // base steps to add to a kernel's step argument to get the absolute step:
  // zero for direct launches, the step at replay start for a captured graph
  // (whose launches carry the steps of its first cycle)
  long long koff;
  double kd[K_N];
  float kf[K_N];
  // state
  void* phi[4];    // R, 1 plane, four buffers (see qb())
  void* sphi[2];   // S, Q-1 planes: f_i - w_i phi, i >= 1 (4 in D2Q5, 8 in D2Q9, 6 in D3Q7)
  void* U[4];      // R, four buffers
  void* jU[2];     // R, dim planes: first moment of the U populations
  void* PU;        // R, pending U increments (accumulated coupling)
  void* T[4];      // R, four buffers
  void* jT[2];     // S, dim planes
  void* PT;        // R
  void* rho[2];    // R
  void* sF[2];     // S, QF-1 planes: f_i - w_i rho, i >= 1 (8 in D2Q9, 18 in D3Q19)
  void* vel[2];    // R, dim planes each
  // variant: grad phi of the phase collision from Eq. (40), lagged one step
  int gradeq40;
  void* gq[2];     // R, 3 planes: v_n dt (x, y) and A = a_s^2 of the last phase step
};

template <class R>
__device__ __forceinline__ R kc(const Dom& d, int i);
template <>
__device__ __forceinline__ double kc<double>(const Dom& d, int i) { return d.kd[i]; }
template <>
__device__ __forceinline__ float kc<float>(const Dom& d, int i) { return d.kf[i]; }

// Per-tile partial reductions written by the kernels (FP64).
struct Partial {
  double solid, M_C, enthalpy, mass;
  double S_phi, J_U;            // max |dU_pc| (transfer), max |injected U|
  double nonfinite;
  double front_max, front_sum;  // 3D: phi = 0 crossing height per column
  double pad;
};

struct DiagOut {
  double solid, M_C, enthalpy, mass, S_phi, J_U;
  double tip[16];
  long long nonfinite;
  long long pad;
};

// Per-XCD work queues of the persistent 2D marching launches: the next
// unclaimed entry of each of the eight lists, one counter per 256-byte line
// (claims on different lists never contend for one line).  Rewound to zero
// by a small kernel before every launch.
constexpr int WQ_LINE = 64;
struct WorkQ {
  unsigned next[8][WQ_LINE];
};
// Runs claimed per atomic.  One run per claim measured fastest on the
// batched ensemble (42.7k MLUPS; 33.7k with two runs, 27.1k with four).
#ifndef LBM_QCHUNK
#define LBM_QCHUNK 1
#endif
constexpr int QCHUNK = LBM_QCHUNK;
// A run list split into eight per-XCD lists: items[qoff[x] .. qoff[x+1]).
struct QList {
  const int4* items;
  const int* qoff;
  int n;
};

// Buffer index holding a field's latest values after `n` writes.
__host__ __device__ inline int par(long long n) { return (int)(n & 1); }

// Buffer index of the phase field, U and T after n writes.  They have four
// buffers, so that a kernel writing the next value may still read the value
// two writes back at sites of other blocks: the kernels that carry a
// deferred transfer read phi^{n-1} (U or T before the transfer) on their
// rings while neighbouring blocks write phi^{n+1} (the transported U or T).
template <class I>
__host__ __device__ inline int qb(I n) { return (int)(n & (I)3); }

// Writes of each buffered plane after completing base step k.  The
// step kernels take k as a 32-bit unsigned step within the cycle of
// 2 lcm(N_chi) base steps, doubled where the write count of phi, U or T
// over it is not a multiple of 4 (every buffer index and every k mod N is
// periodic with it), so their divisions are 32-bit; the host and the
// read-out kernels use the absolute 64-bit step.
template <class I>
__host__ __device__ inline I n_phi(const Dom& d, I k) { return k / (I)d.N_phi; }
template <class I>
__host__ __device__ inline I n_U(const Dom& d, I k) {
  return (d.accum ? I(0) : k / (I)d.N_phi) + k / (I)d.N_U;
}
template <class I>
__host__ __device__ inline I n_jU(const Dom& d, I k) { return k / (I)d.N_U; }
// T is written, like U, by the transfer of every phase step (latent heat,
// instantaneous coupling) and by its own transport; its first moment only
// by the transport
template <class I>
__host__ __device__ inline I n_Ttr(const Dom& d, I k) {
  return (d.has_T && !d.accum && !d.T_pulled) ? k / (I)d.N_phi : I(0);
}
template <class I>
__host__ __device__ inline I n_T(const Dom& d, I k) { return n_Ttr(d, k) + k / (I)d.N_T; }
template <class I>
__host__ __device__ inline I n_jT(const Dom& d, I k) { return k / (I)d.N_T; }
template <class I>
__host__ __device__ inline I n_F(const Dom& d, I k) { return k / (I)d.N_F; }

}  // namespace lbm
