// Host runtime and C ABI of the multirate lattice-Boltzmann library.
//
// A context owns one workspace (caller-supplied or allocated here) carved into
// the per-domain state planes, the device descriptors, the tile lists and the
// reduction buffers.  Stepping issues, per base step k, the kernels whose
// field is due (k mod N_chi == 0, Eq. 34) in the order phase, transfer, U, T,
// flow; whole cycles of 2 * lcm(N_chi) base steps, or twice that (the
// period after which every buffer index repeats: parities of the
// double-buffered planes, write counts mod 4 of phi, U and T), are captured
// once into a HIP graph and replayed.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_dev.h"

namespace lbm {
template <class R, class S>
struct Launch {
  static void phase(int TY, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k);
  static void transfer(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p);
  static int phase_tr_rows(int TY);
  static void phase_tr(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p);
  static void phase_ym(int Q, dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k);
  static void phase_ymq(int Q, const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k);
  static void transfer_ymq(const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k, double2* rmax);
  static void scalar_ymq(int field, int Q, const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k,
                         double2* rmax);
  static void tr_scalar_ymq(int Q, const QList& l, WorkQ* q, hipStream_t st, const Dom* d, unsigned k,
                            double2* rmax);
  static void dtr_phase(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p);
  static void dtr_scalar(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k, Partial* p);
  static void transfer_ym(dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k, double2* rmax);
  static void tr_scalar_ym(int Q, dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k,
                           double2* rmax);
  static void scalar_ym(int field, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* runs, unsigned k,
                        double2* rmax);
  static void scalar(int field, int TY, int Q, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k,
                     Partial* p);
  static void flow(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, unsigned k);
  static void diag_tiles(int TY, dim3 g, hipStream_t st, const Dom* d, const int4* t, long long k, Partial* p);
  static void tips(int ndom, hipStream_t st, const Dom* d, long long k, DiagOut* o);
  static void init(hipStream_t st, const Dom* d, int dom, long long n, const double* xi);
  static void read(hipStream_t st, const Dom* d, int dom, long long k, const int* codes, int nc, int f64,
                   void* out, long long n);
  static void write(hipStream_t st, const Dom* d, int dom, long long k, const int* codes, int nc,
                    const double* src, long long n);
};
void diag_final(int ndom, hipStream_t st, const Dom* d, const Partial* p, const int* slot, const int* slot0,
                const double2* rmax, int src, DiagOut* o);
void nonfinite_check(int f64, int ndom, int blocks, hipStream_t st, const Dom* d, long long k,
                     unsigned long long* first);
template <class R, class S>
struct Launch3 {
  static void phase(const Dom& h, hipStream_t st, const Dom* d, unsigned k, int rows, int zblk);
  static void transfer(const Dom& h, hipStream_t st, const Dom* d, unsigned k, Partial* p, int rows, int zblk);
  static void scalar(int field, const Dom& h, hipStream_t st, const Dom* d, unsigned k, Partial* p, int rows,
                     int zblk);
  static void flow(const Dom& h, hipStream_t st, const Dom* d, unsigned k, int rows, int zblk);
  static void step(const Dom& h, hipStream_t st, const Dom* d, unsigned k, Partial* p, const int* rows,
                   const int* zblk);
  static void init(const Dom& h, hipStream_t st, const Dom* d, const double* xi);
  static void diag(const Dom& h, hipStream_t st, const Dom* d, long long k, Partial* p, double* front);
  static void read(const Dom& h, hipStream_t st, const Dom* d, long long k, const int* codes, int nc, int f64,
                   void* out);
  static void write(const Dom& h, hipStream_t st, const Dom* d, long long k, const int* codes, int nc,
                    const double* src);
  static void set_koff(hipStream_t st, Dom* d, long long koff);
};
}  // namespace lbm

using namespace lbm;

namespace {

constexpr int kNTY = 4;
constexpr int kTYs[kNTY] = {4, 8, 16, 32};
constexpr long long kMaxGraphSteps = 4096;
constexpr int kMaxCodes = 96;
constexpr int kStagePlanes = 20;   // host staging planes: holds one D3Q19 population group

std::string g_create_error;

struct TileSet {
  int4* d = nullptr;  // device list (XCD-ordered, padded to a multiple of 8)
  int n = 0;          // padded length = grid size
};

struct Group {
  int N;              // update factor shared by the domains of the group
  TileSet ts[kNTY];   // per tile height
  TileSet runs;       // column runs, YCOL wide and YRUN rows high (2D marching kernels)
  TileSet runs64;     // phase field: runs 64 wide (the marching phase kernel)
  QList q, q64;       // the same runs as eight per-XCD work-queue lists
};

struct Ops {
  void (*phase)(int, int, dim3, hipStream_t, const Dom*, const int4*, unsigned);
  void (*transfer)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned, Partial*);
  void (*phase_tr)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned, Partial*);
  int (*phase_tr_rows)(int);
  void (*phase_ym)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned);
  void (*phase_ymq)(int, const QList&, WorkQ*, hipStream_t, const Dom*, unsigned);
  void (*transfer_ymq)(const QList&, WorkQ*, hipStream_t, const Dom*, unsigned, double2*);
  void (*scalar_ymq)(int, int, const QList&, WorkQ*, hipStream_t, const Dom*, unsigned, double2*);
  void (*tr_scalar_ymq)(int, const QList&, WorkQ*, hipStream_t, const Dom*, unsigned, double2*);
  void (*dtr_phase)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned, Partial*);
  void (*dtr_scalar)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned, Partial*);
  void (*transfer_ym)(dim3, hipStream_t, const Dom*, const int4*, unsigned, double2*);
  void (*tr_scalar_ym)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned, double2*);
  void (*scalar_ym)(int, int, dim3, hipStream_t, const Dom*, const int4*, unsigned, double2*);
  void (*scalar)(int, int, int, dim3, hipStream_t, const Dom*, const int4*, unsigned, Partial*);
  void (*flow)(int, dim3, hipStream_t, const Dom*, const int4*, unsigned);
  void (*diag_tiles)(int, dim3, hipStream_t, const Dom*, const int4*, long long, Partial*);
  void (*tips)(int, hipStream_t, const Dom*, long long, DiagOut*);
  void (*init)(hipStream_t, const Dom*, int, long long, const double*);
  void (*read)(hipStream_t, const Dom*, int, long long, const int*, int, int, void*, long long);
  void (*write)(hipStream_t, const Dom*, int, long long, const int*, int, const double*, long long);
};

template <class R, class S>
Ops make_ops() {
  return Ops{Launch<R, S>::phase, Launch<R, S>::transfer, Launch<R, S>::phase_tr, Launch<R, S>::phase_tr_rows,
             Launch<R, S>::phase_ym, Launch<R, S>::phase_ymq, Launch<R, S>::transfer_ymq, Launch<R, S>::scalar_ymq,
             Launch<R, S>::tr_scalar_ymq, Launch<R, S>::dtr_phase, Launch<R, S>::dtr_scalar, Launch<R, S>::transfer_ym, Launch<R, S>::tr_scalar_ym, Launch<R, S>::scalar_ym, Launch<R, S>::scalar, Launch<R, S>::flow,
             Launch<R, S>::diag_tiles, Launch<R, S>::tips, Launch<R, S>::init, Launch<R, S>::read,
             Launch<R, S>::write};
}

struct Ops3 {
  void (*phase)(const Dom&, hipStream_t, const Dom*, unsigned, int, int);
  void (*transfer)(const Dom&, hipStream_t, const Dom*, unsigned, Partial*, int, int);
  void (*scalar)(int, const Dom&, hipStream_t, const Dom*, unsigned, Partial*, int, int);
  void (*flow)(const Dom&, hipStream_t, const Dom*, unsigned, int, int);
  void (*step)(const Dom&, hipStream_t, const Dom*, unsigned, Partial*, const int*, const int*);
  void (*init)(const Dom&, hipStream_t, const Dom*, const double*);
  void (*diag)(const Dom&, hipStream_t, const Dom*, long long, Partial*, double*);
  void (*read)(const Dom&, hipStream_t, const Dom*, long long, const int*, int, int, void*);
  void (*write)(const Dom&, hipStream_t, const Dom*, long long, const int*, int, const double*);
  void (*set_koff)(hipStream_t, Dom*, long long);
};

template <class R, class S>
Ops3 make_ops3() {
  return Ops3{Launch3<R, S>::phase, Launch3<R, S>::transfer, Launch3<R, S>::scalar, Launch3<R, S>::flow,
              Launch3<R, S>::step,  Launch3<R, S>::init,     Launch3<R, S>::diag,   Launch3<R, S>::read,
              Launch3<R, S>::write, Launch3<R, S>::set_koff};
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

long long ipow_lcm(long long a, long long b) { return a / std::gcd(a, b) * b; }

}  // namespace

// Reduction scratch of the step and diagnostics kernels: per-tile (3D:
// per-block) partials, per-run maxima of the marching kernels, the reduced
// diagnostics and the 3D front partials.  The workspace holds one set; the
// allocation-free entry point carves another from a static device array.
struct Scratch {
  Partial* part = nullptr;
  double2* rmax = nullptr;   // per marching run: largest |dU| and injected U of the last transfer
  DiagOut* diag = nullptr;
  double* front = nullptr;   // 3D front partials: (max, sum) per column block
};

struct lbm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int storage = LBM_STORE_F32;
  size_t rsz = 4, ssz = 4;
  Ops ops{};
  Ops3 ops3{};
  int dim = 2;
  long long koff = 0;           // value of Dom::koff on the device (3D)
  int nfront = 0;
  Scratch s;                   // the set the kernels use: ws_s, or the static one during a static call
  Scratch ws_s;                // the workspace's set
  size_t scratch_bytes = 0;    // bytes of one set (the static array must hold them)
  long long nparts = 0, nrmax = 0;
  // pinned host staging for the diagnostics, allocated at creation
  DiagOut* h_diag = nullptr;
  unsigned long long* h_first = nullptr;
  double* h_front = nullptr;
  std::vector<lbm_diag> h_d;
  int nblk3 = 0;               // 3D: site blocks of 256
  int ndom = 0;
  std::vector<lbm_params> P;
  std::vector<Dom> H;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  Dom* d_dom = nullptr;
  TileSet all[kNTY];
  std::vector<Group> g_phi, g_U, g_T, g_F;
  int* d_slot = nullptr;
  bool tr_march = false;       // the last launched transfer marched (the diagnostics read d_rmax)
  bool u_march = false;        // the last launched U transport marched (accumulated J_U in d_rmax)
  unsigned long long* d_first = nullptr;   // per domain: first checked step with a non-finite value
  int nf_blocks = 1;           // grid width of the non-finite screen
  std::vector<double> m0;      // M_C at the start of the run (for R_M)
  bool need_m0 = true;         // M_C(0) is taken at the first step after an initialisation
  int* d_slot0[kNTY] = {nullptr, nullptr, nullptr, nullptr};
  int* d_codes = nullptr;
  double* d_stage = nullptr;
  size_t stage_elems = 0;
  int ty_index = 2;
  bool tuned = false;
  bool autotune = true;
  bool use_graph = true;
  bool fuse = false;      // phase + transfer in one kernel (2D) when every domain allows it
  bool fusable = false;   // every domain at least 8 x 8 (the fused kernel's rings wrap once at most), D2Q5
  int march = 0;          // 2D marching phase kernel: 0 by size, 1 always, -1 never
  bool defer = true;      // defer a phase step's transfer into the next phase kernel where allowed
  bool deferrable = false;// D2Q5, one phase group with N_phi = 1, instantaneous coupling, domains >= 8 x 8
  bool pending = false;   // the last launched step's transfer is deferred
  bool one_U = false;     // every domain has U, all in one update group
  bool one_T = false;     // one phase group; every domain has a transported T, all in one update group
  bool march_big = false; // the phase groups hold enough column runs to fill the chip
  bool marchable = false; // every domain 2D and at least 16 x 16 (the marching windows wrap once at most)
  bool march_pick = false; // marching or tiles by the size rule (march_big); lbm_configure can force either
  int queue = 0;          // marching launches: 0 autotuned, 1 per-XCD work queues, -1 static grids
  bool use_q = false;     // the marching kernels run from the work queues
  int rows3 = 0;          // 3D tile rows of every kernel: 4, 8, or 0 for the per-kernel choice
  int rows3k[5] = {0, 0, 0, 0, 0};   // 3D per-kernel tile rows (0: the default) ...
  int zblk3k[5] = {0, 0, 0, 0, 0};   // ... and z-run block targets, as the autotuner picked them
  WorkQ* d_wq = nullptr;  // the queues' counters (rewound before each launch)
  int qs = 5;             // scalar lattice of the (2D) context: 5 or 9
  hipGraphExec_t gexec = nullptr;
  int graph_ty = -1;
  long long cycle = 1;
  long long k = 0;
  std::vector<bool> initialised;
  std::string err;
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& m) {
  if (c)
    c->err = m;
  else
    g_create_error = m;
  return s;
}

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(ctx, LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

int px_of(int nx) { return (nx + 63) / 64 * 64; }

// elements per plane and the per-domain byte layout
struct Layout {
  size_t rplanes = 0, splanes = 0;
};

Layout layout_of(const lbm_params& p) {
  Layout L;
  const int d = p.dim;
  L.rplanes = 4;                           // phi, four buffers
  L.splanes = 2 * (p.q_scalar - 1);        // phase s_i, two buffers
  if (p.has_U) L.rplanes += 5 + 2 * d;                    // U (four buffers), pending U, first moment
  if (p.has_T) { L.rplanes += 5; L.splanes += 2 * d; }   // T (four buffers), pending T
  if (p.has_flow) { L.rplanes += 2 + 2 * d; L.splanes += 2 * (d == 3 ? 18 : 8); }
  if (p.grad_phi == 1) L.rplanes += 6;   // Eq. (40) variant: v_n dt and A, two buffers
  return L;
}

long long sites_of(const lbm_params& p) { return (long long)p.nx * p.ny * (p.dim == 3 ? p.nz : 1); }
// 3D grid: one block per 64 x 4 tile of a z plane, tile columns padded to a
// multiple of the 8 XCDs (the mapping of the 3D kernels)
long long blocks3(const lbm_params& p) {
  const long long cols = (long long)((p.nx + 63) / 64) * ((p.ny + 3) / 4);
  return (cols + 7) / 8 * 8 * p.nz;
}

size_t sizes_of(int storage, size_t& rsz, size_t& ssz) {
  rsz = storage == LBM_STORE_F64 ? 8 : 4;
  ssz = storage == LBM_STORE_F64 ? 8 : storage == LBM_STORE_F32 ? 4 : 2;
  return 0;
}

std::string validate(const lbm_params& p, int i) {
  char b[256];
  auto bad = [&](const char* m) {
    snprintf(b, sizeof b, "domain %d: %s", i, m);
    return std::string(b);
  };
  if (p.dim != 2 && p.dim != 3) return bad("dim must be 2 or 3");
  if (p.dim == 2 && p.nz != 1) return bad("nz must be 1 in 2D");
  if (p.nx < 3 || p.ny < 3 || p.nx > (1 << 16) || p.ny > (1 << 16)) return bad("grid sides must be in [3, 65536]");
  if (p.dim == 3 && (p.nz < 3 || p.nz > (1 << 16))) return bad("nz must be in [3, 65536]");
  // in-plane offsets (up to 18 planes apart) are 32-bit unsigned in the kernels
  if ((long long)((p.nx + 63) / 64 * 64) * p.ny * (p.dim == 3 ? p.nz : 1) > (1LL << 27))
    return bad("more than 2^27 sites in one domain");
  if (p.dim == 2 && p.q_scalar != 5 && p.q_scalar != 9)
    return bad("2D scalar lattice must be D2Q5 or D2Q9 (q_scalar = 5 or 9)");
  if (p.dim == 3 && p.q_scalar != 7) return bad("3D scalar lattice must be D3Q7 (q_scalar = 7)");
  if (p.dim == 3) {
    for (int a = 0; a < 3; ++a)
      if (p.flow_bc[a] == LBM_BC_INLET_OUTFLOW) return bad("inlet/outflow is 2D only");
    if (p.bc[2] != LBM_BC_PERIODIC && p.bc[2] != LBM_BC_WALL) return bad("bad z boundary");
    if (p.has_flow && p.u0_liquid_only) return bad("3D flow starts at rest (u0_liquid_only is 2D only)");
  }
  if (p.T_mode != LBM_T_TRANSPORT && p.T_mode != LBM_T_PULLED && p.T_mode != LBM_T_DIRICHLET_LOW)
    return bad("bad T_mode");
  if (p.T_mode == LBM_T_DIRICHLET_LOW && p.bc[p.dim - 1] != LBM_BC_WALL)
    return bad("the cold bottom needs walls on the last axis");
  if (p.T_mode == LBM_T_PULLED && (p.dim != 3 || p.bc[2] != LBM_BC_WALL))
    return bad("the pulled temperature needs a 3D domain with z walls");
  if (p.T_mode == LBM_T_PULLED && (p.kappa_S != p.kappa_L || p.rhoCp_S != p.rhoCp_L))
    return bad("the pulled temperature needs constant thermal properties");
  if (p.N_phi < 1 || p.N_U < 1 || p.N_T < 1 || p.N_F < 1) return bad("update factors must be >= 1");
  if (!(p.dt_base > 0)) return bad("dt_base must be > 0");
  if (!(p.W0 > 0) || !(p.tau0 > 0)) return bad("W0 and tau0 must be > 0");
  if (p.eps_s < 0 || p.eps_s >= 0.25) return bad("eps_s must be in [0, 0.25)");
  for (int a = 0; a < 2; ++a) {
    if (p.bc[a] != LBM_BC_PERIODIC && p.bc[a] != LBM_BC_WALL) return bad("scalar bc must be periodic or wall");
    if (p.flow_bc[a] < 0 || p.flow_bc[a] > 2) return bad("bad flow bc");
  }
  if (p.flow_bc[1] == LBM_BC_INLET_OUTFLOW) return bad("inlet/outflow is supported along x only");
  if (p.coupling != LBM_COUPLE_INSTANT && p.coupling != LBM_COUPLE_ACCUM) return bad("bad coupling");
  if (p.grad_phi != LBM_GRAD_ISO && p.grad_phi != LBM_GRAD_EQ40) return bad("bad grad_phi");
  if (p.grad_phi == LBM_GRAD_EQ40 && p.dim != 2) return bad("the Eq. (40) phase gradient is 2D only");
  // relaxation times at phi = +-1 (Eq. 24, 32): every tau must exceed 1/2
  const double amin = 1.0 - 5.0 / 3.0 * p.eps_s;
  const double ics2 = p.dim == 3 ? 4.0 : 3.0;   // 1/c_s^2 of the scalar lattice
  const double tphi = ics2 * p.N_phi * p.dt_base * amin * amin * p.W0 * p.W0 / p.tau0 + 0.5;
  if (!(tphi > 0.5)) return bad("tau_phi <= 1/2");
  if (p.has_U) {
    for (double ph : {-1.0, 1.0}) {
      const double kf = (1 + p.k) - (1 - p.k) * ph;
      if (!(kf > 0)) return bad("(1+k) - (1-k) phi must be > 0");
      const double De = ((1 + ph) * p.D_S + (1 - ph) * p.D_L) / kf;
      if (!(ics2 * p.N_U * p.dt_base * De + 0.5 > 0.5)) return bad("tau_U <= 1/2");
    }
  }
  if (p.has_T) {
    if (!(p.rhoCp_S > 0) || !(p.rhoCp_L > 0)) return bad("rhoCp must be > 0");
    for (double ph : {-1.0, 1.0}) {
      const double a = ((1 + ph) / 2 * p.kappa_S + (1 - ph) / 2 * p.kappa_L) /
                       ((1 + ph) / 2 * p.rhoCp_S + (1 - ph) / 2 * p.rhoCp_L);
      if (!(ics2 * p.N_T * p.dt_base * a + 0.5 > 0.5)) return bad("tau_T <= 1/2");
    }
    if (!(p.L_h != 0) || !(p.Cp_L > 0)) return bad("L_h and Cp_L must be nonzero");
  }
  if (p.has_flow && !(3.0 * p.N_F * p.dt_base * p.nu + 0.5 > 0.5)) return bad("tau_F <= 1/2");
  return "";
}

// XCD-aware tile list: spatial tiles s = 0..n-1 (domain-major, row-major)
// are split into 8 contiguous chunks, chunk x going to the blocks b with
// b mod 8 == x (workgroups are dispatched round-robin over the eight XCDs),
// so neighbouring tiles share an XCD's L2 and halo re-reads hit it.
std::vector<int4> xcd_order(const std::vector<int4>& spatial) {
  const int n = (int)spatial.size();
  const int c = (n + 7) / 8;
  std::vector<int4> out((size_t)8 * c, make_int4(-1, 0, 0, 0));
  for (int b = 0; b < 8 * c; ++b) {
    const int s = (b % 8) * c + b / 8;
    if (s < n) out[b] = spatial[s];
  }
  return out;
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Scratch of lbm_step_multirate_static, for callers that cannot allocate:
// one array per device, held until the process ends.  Its name is a host
// stand-in in host code; kernels get the device address that
// hipGetSymbolAddress returns on each device, taken once per device with
// that device current (at the first lbm_create on it).
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};
static hipError_t g_scratch_err[kMaxDevices] = {};
static bool g_scratch_done[kMaxDevices] = {};

// clears a range of the static scratch (a kernel, so that no memset node
// lands in a caller's captured graph)
__global__ void k_zero_words(unsigned long long* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

static void static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
  g_scratch_done[device] = true;
}

// ------------------------------------------------------------------ helpers
static int ty_slot(int rows) {
  for (int i = 0; i < kNTY; ++i)
    if (kTYs[i] == rows) return i;
  return 0;
}

// The step kernels take the base step within the cycle: absolute step k >= 1
// maps to 1 + (k - 1) mod cycle, which keeps every k mod N_chi and every
// buffer index, so their index arithmetic stays 32-bit.  The
// time-dependent 3D walls add Dom::koff, the absolute step at the start of
// the cycle.
static unsigned cycle_step(const lbm_ctx* c, long long k) { return (unsigned)((k - 1) % c->cycle + 1); }

// whether the phase field runs on the marching kernel
static bool use_march(const lbm_ctx* c) {
  return c->marchable && (c->march > 0 || (c->march == 0 && c->march_pick));
}

// Whether the transfer of phase step k (within the cycle) waits for the
// phase kernel of step k + 1: no transport runs at step k, k is not the
// cycle's last step, and the context allows it.
static bool defers(const lbm_ctx* c, unsigned k) {
  if (!(c->defer && c->deferrable && !c->fuse && !use_march(c)) || (long long)k >= c->cycle) return false;
  for (auto* gs : {&c->g_U, &c->g_T, &c->g_F})
    for (auto& g : *gs)
      if (k % g.N == 0) return false;
  return true;
}

// Whether the transfer of phase step k runs inside the U transport of step
// k: the U update is due at k, every domain has U in one update group, and
// the context allows deferred transfers.
static bool fuses_U(const lbm_ctx* c, unsigned k) {
  if (!(c->defer && c->deferrable && c->one_U && !c->fuse && !use_march(c))) return false;
  return k % c->g_U[0].N == 0;
}

// Whether the marching transfer of phase step k runs inside the T
// transport of step k: both are due at k, every domain has a transported
// T with instantaneous coupling in one update group, and the context
// allows deferred transfers.
static bool fuses_T(const lbm_ctx* c, unsigned k) {
  if (!(c->defer && c->one_T && !c->fuse && use_march(c))) return false;
  return k % c->g_T[0].N == 0 && k % c->g_phi[0].N == 0;
}

// 3D tile rows per kernel kind (0 phase, 1 transfer, 2 U, 3 T, 4 flow):
// those fixed by lbm_configure, else the autotuner's pick (phase, transfer,
// U transport, flow), else the height measured best on the 256 x 256 x 512
// directional workload (the flow's LDS window allows 8 rows with FP32
// arithmetic only).  ms per launch at 4 / 8 rows, each at its best z runs:
// phase 0.433 / 0.363, transfer 0.228 / 0.216, U 0.418 / 0.376, T 0.338 /
// 0.284, flow 1.198 / 1.132
constexpr int kRows3Default[5] = {8, 8, 8, 8, 8};
// z-run lengths: each kernel's runs aim at this many blocks of 256 threads
// (half as many of 512), the fastest of 512 ... 8192 on the same workload
// (ms per launch at 1024 / 1536 / 2048 / 3072 / 4096 / 8192, 8 rows: phase
// 0.384 / 0.363 / 0.399 / 0.368 / 0.374 / 0.379 (1536: one round of three
// blocks per CU), transfer 0.247 / 0.216 / 0.262 / 0.222 / 0.224 / 0.233,
// flow 1.132 / 1.142 / 1.158 / 1.185 / 1.196 / 1.269, U transport 0.396 /
// 0.376 / 0.428 / 0.388 / 0.399 / 0.405; T at 1536 / 3072 / 4096 / 8192
// 0.294 / 0.280 / 0.276 / 0.272)
constexpr int kZBlocks3[5] = {1536, 1536, 1536, 8192, 1024};
static int rows3(const lbm_ctx* c, int kind) {
  const int r = c->rows3 != 0 ? c->rows3 : c->rows3k[kind] != 0 ? c->rows3k[kind] : kRows3Default[kind];
  return kind == 4 && c->storage == LBM_STORE_F64 ? 4 : r;
}
static int zblk3(const lbm_ctx* c, int kind) { return c->zblk3k[kind] != 0 ? c->zblk3k[kind] : kZBlocks3[kind]; }

static void launch_step(lbm_ctx* c, hipStream_t st, unsigned k, bool last = false) {
  if (c->dim == 3) {
    const int rows[5] = {rows3(c, 0), rows3(c, 1), rows3(c, 2), rows3(c, 3), rows3(c, 4)};
    const int zblk[5] = {zblk3(c, 0), zblk3(c, 1), zblk3(c, 2), zblk3(c, 3), zblk3(c, 4)};
    c->ops3.step(c->H[0], st, c->d_dom, k, c->s.part, rows, zblk);
    return;
  }
  const int ti = c->ty_index, TY = kTYs[ti];
  const bool fused = c->fuse && c->fusable;
  const int tf = fused ? ty_slot(c->ops.phase_tr_rows(TY)) : ti;
  for (auto& g : c->g_phi)
    if (k % g.N == 0) {
      c->tr_march = !fused && use_march(c);
      if (fused) {
        c->ops.phase_tr(kTYs[tf], dim3(g.ts[tf].n), st, c->d_dom, g.ts[tf].d, k, c->s.part);
      } else {
        if (use_march(c)) {
          if (c->use_q) c->ops.phase_ymq(c->qs, g.q64, c->d_wq, st, c->d_dom, k);
          else c->ops.phase_ym(c->qs, dim3(g.runs64.n), st, c->d_dom, g.runs64.d, k);
          if (!fuses_T(c, k)) {   // else inside the T transport, launched first below
            if (c->use_q) c->ops.transfer_ymq(g.q, c->d_wq, st, c->d_dom, k, c->s.rmax);
            else c->ops.transfer_ym(dim3(g.runs.n), st, c->d_dom, g.runs.d, k, c->s.rmax);
          }
        } else {
          if (c->pending)   // the previous step's transfer runs inside this phase kernel
            c->ops.dtr_phase(TY, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k, c->s.part);
          else
            c->ops.phase(TY, c->qs, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k);
          c->pending = !last && defers(c, k);
          if (!c->pending && !fuses_U(c, k))   // else in the phase kernel of step k + 1 or the U transport
            c->ops.transfer(TY, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k, c->s.part);
        }
      }
    }
  const bool march = use_march(c);
  // the transfer fused into the T transport precedes the U transport, which
  // reads the transferred U (the two transports are independent)
  const bool trT = fuses_T(c, k);
  if (trT)
    for (auto& g : c->g_T) {
      if (c->use_q) c->ops.tr_scalar_ymq(c->qs, g.q, c->d_wq, st, c->d_dom, k, c->s.rmax);
      else c->ops.tr_scalar_ym(c->qs, dim3(g.runs.n), st, c->d_dom, g.runs.d, k, c->s.rmax);
    }
  // (the U transport marches too since the runs are 62 columns wide: 191
  // against 224 us per launch on the batched ensemble)
  for (auto& g : c->g_U)
    if (k % g.N == 0) {
      c->u_march = march && !fuses_U(c, k);
      if (fuses_U(c, k))   // carrying this step's transfer
        c->ops.dtr_scalar(TY, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k, c->s.part);
      else if (march && c->use_q)
        c->ops.scalar_ymq(0, c->qs, g.q, c->d_wq, st, c->d_dom, k, c->s.rmax);
      else if (march)
          c->ops.scalar_ym(0, c->qs, dim3(g.runs.n), st, c->d_dom, g.runs.d, k, c->s.rmax);
        else
          c->ops.scalar(0, TY, c->qs, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k, c->s.part);
    }
  for (auto& g : c->g_T)
    if (k % g.N == 0 && !trT) {
      if (march && c->use_q) c->ops.scalar_ymq(1, c->qs, g.q, c->d_wq, st, c->d_dom, k, c->s.rmax);
      else if (march) c->ops.scalar_ym(1, c->qs, dim3(g.runs.n), st, c->d_dom, g.runs.d, k, c->s.rmax);
      else c->ops.scalar(1, TY, c->qs, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k, c->s.part);
    }
  for (auto& g : c->g_F)
    if (k % g.N == 0) c->ops.flow(TY, dim3(g.ts[ti].n), st, c->d_dom, g.ts[ti].d, k);
}

static lbm_status upload_doms(lbm_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->d_dom, c->H.data(), sizeof(Dom) * c->ndom, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// Time each tile height on the kernels whose launches are idempotent for a
// fixed k (they read one buffer and write the other: the phase kernel, or
// the phase + transfer kernel with instantaneous coupling, and the flow)
// and keep the fastest.  The tiled phase kernel is timed also when the
// phase field marches: it then stands in for the tiled transfer and
// transports, which share its tile shape and access pattern.
static lbm_status autotune(lbm_ctx* c) {
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float best = 1e30f;
  int besti = 1;
  bool any_accum = false;
  for (auto& D : c->H) any_accum |= D.accum != 0;
  // the next due step of a group: its kernels read the current buffers and
  // write only the other ones, so repeating them leaves the state unchanged
  auto next_due = [&](int N) { return cycle_step(c, (c->k / N + 1) * (long long)N); };
  for (int ti = 0; ti < kNTY; ++ti) {
    const int TY = kTYs[ti];
    auto run = [&]() {
      const bool fused = c->fuse && c->fusable && !any_accum;   // accumulated coupling adds in place
      const int tf = fused ? ty_slot(c->ops.phase_tr_rows(TY)) : ti;
      for (auto& g : c->g_phi) {
        if (fused)
          c->ops.phase_tr(kTYs[tf], dim3(g.ts[tf].n), c->stream, c->d_dom, g.ts[tf].d, next_due(g.N), nullptr);
        else
          c->ops.phase(TY, c->qs, dim3(g.ts[ti].n), c->stream, c->d_dom, g.ts[ti].d, next_due(g.N));
      }
      // (the U and T transports are not timed: with instantaneous coupling
      // the transfer of the same step also writes their planes, so the
      // transport of the next due step writes the current buffer; with
      // accumulated coupling it clears the pending planes)
      for (auto& g : c->g_F) c->ops.flow(TY, dim3(g.ts[ti].n), c->stream, c->d_dom, g.ts[ti].d, next_due(g.N));
    };
    run();
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < 5; ++r) run();
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      besti = ti;
    }
  }
  c->ty_index = besti;
  // marching contexts: static grids or the per-XCD work queues, timed on
  // the marching phase kernel (the other marching kernels follow the pick)
  if (c->marchable && use_march(c) && c->queue == 0 && !(c->fuse && c->fusable)) {
    float t2[2] = {0.f, 0.f};
    for (int form = 0; form < 2; ++form) {
      auto run = [&]() {
        for (auto& g : c->g_phi) {
          if (form) c->ops.phase_ymq(c->qs, g.q64, c->d_wq, c->stream, c->d_dom, next_due(g.N));
          else c->ops.phase_ym(c->qs, dim3(g.runs64.n), c->stream, c->d_dom, g.runs64.d, next_due(g.N));
        }
      };
      run();
      HIPCHK(c, hipEventRecord(e0, c->stream));
      for (int r = 0; r < 5; ++r) run();
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      HIPCHK(c, hipEventElapsedTime(&t2[form], e0, e1));
    }
    c->use_q = t2[1] < t2[0];
  }
  HIPCHK(c, hipEventDestroy(e0));
  HIPCHK(c, hipEventDestroy(e1));
  c->tuned = true;
  return LBM_OK;
}

// 3D: time each of the phase kernel, the flow and (with N_phi = 1 and
// instantaneous coupling) the transfer at both tile heights and four z-run
// block targets, on launches that leave the state unchanged (at the next
// due step they read the current buffers and write only the next ones),
// and keep the fastest for each.  The U and T transports keep the measured
// defaults: at their next due step they would write a current buffer (the
// transfer of that step has not run) or clear the pending planes.  The
// transfer's partials are cleared afterwards.
static lbm_status autotune3(lbm_ctx* c) {
  const Dom& h = c->H[0];
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  auto next_due = [&](int N) { return cycle_step(c, (c->k / N + 1) * (long long)N); };
  const bool f64 = c->storage == LBM_STORE_F64;
  const bool tr_ok = h.N_phi == 1 && !h.accum;
  // the U transport of the next step reads the transfer's output buffer
  // (not yet written) and writes a buffer two updates old, which that step
  // overwrites again: it can be timed in place when U and phi advance
  // together with instantaneous coupling
  const bool u_ok = tr_ok && h.has_U && h.N_U == 1;
  // z-run block targets: 1536 and 3072 fill the chip in one and two rounds
  // of 64 x 8 blocks at three blocks per CU
  constexpr int NZ = 6;
  const int zs[NZ] = {1024, 1536, 2048, 3072, 4096, 8192};
  const bool log = std::getenv("LBM_AUTOTUNE_LOG") != nullptr;
  for (int kind : {0, 1, 2, 4}) {
    if (kind == 1 && !tr_ok) continue;
    if (kind == 2 && !u_ok) continue;
    if (kind == 4 && !h.has_F) continue;
    auto time_of = [&](int rows, int z) -> float {
      auto run = [&]() {
        if (kind == 0) c->ops3.phase(h, c->stream, c->d_dom, next_due(h.N_phi), rows, z);
        if (kind == 1) c->ops3.transfer(h, c->stream, c->d_dom, next_due(h.N_phi), c->s.part, rows, z);
        if (kind == 2) c->ops3.scalar(0, h, c->stream, c->d_dom, next_due(h.N_U), c->s.part, rows, z);
        if (kind == 4) c->ops3.flow(h, c->stream, c->d_dom, next_due(h.N_F), rows, z);
      };
      run();
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < 3; ++r) run();
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      return hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? ms : 1e30f;
    };
    // every choice is timed in two passes and keeps its faster time (the
    // first launches of a context run while the clocks still ramp up); the
    // measured default stands unless another choice is faster by more than
    // 2 % (the spread of repeated timings)
    const int r0 = (kind == 4 && f64) ? 4 : kRows3Default[kind], z0 = kZBlocks3[kind];
    float t[2][NZ];
    for (int pass = 0; pass < 2; ++pass)
      for (int ri = 0; ri < 2; ++ri)
        for (int zi = 0; zi < NZ; ++zi) {
          const bool skip = kind == 4 && ri == 1 && f64;
          const float ms = skip ? 1e30f : time_of(4 + 4 * ri, zs[zi]);
          t[ri][zi] = pass == 0 ? ms : std::min(t[ri][zi], ms);
        }
    float best = 1e30f;
    for (int zi = 0; zi < NZ; ++zi)
      if (zs[zi] == z0) best = t[r0 == 8 ? 1 : 0][zi];
    c->rows3k[kind] = r0;
    c->zblk3k[kind] = z0;
    for (int ri = 0; ri < 2; ++ri)
      for (int zi = 0; zi < NZ; ++zi)
        if (t[ri][zi] < 0.98f * best) {
          best = t[ri][zi];
          c->rows3k[kind] = 4 + 4 * ri;
          c->zblk3k[kind] = zs[zi];
        }
    if (log) {   // ms per launch (three launches), then the pick
      for (int ri = 0; ri < 2; ++ri) {
        std::fprintf(stderr, "lbm autotune3 kind %d rows %d:", kind, 4 + 4 * ri);
        for (int zi = 0; zi < NZ; ++zi) std::fprintf(stderr, " %d=%.4f", zs[zi], t[ri][zi] / 3.0f);
        std::fprintf(stderr, "\n");
      }
      std::fprintf(stderr, "lbm autotune3 kind %d pick rows %d z-blocks %d\n", kind, c->rows3k[kind],
                   c->zblk3k[kind]);
    }
    HIPCHK(c, hipGetLastError());
  }
  HIPCHK(c, hipMemsetAsync(c->ws_s.part, 0, sizeof(Partial) * (size_t)c->nparts, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipEventDestroy(e0));
  HIPCHK(c, hipEventDestroy(e1));
  c->tuned = true;
  return LBM_OK;
}

// ------------------------------------------------------------------ ABI
extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p, int32_t n, int32_t storage) {
  if (!p || n < 1 || storage < 0 || storage > 3) return 0;
  size_t rsz, ssz;
  sizes_of(storage, rsz, ssz);
  size_t total = 0;
  long long tilesmax = 0;   // tiles at the smallest tile height
  long long runs = 0;       // column runs of the 2D marching kernels
  size_t maxsites = 0;
  for (int i = 0; i < n; ++i) {
    if (!validate(p[i], i).empty()) return 0;
    if (p[i].dim == 2)
      runs += (long long)((p[i].nx + YCOL - 1) / YCOL + (p[i].nx + 63) / 64) * ((p[i].ny + YRUN - 1) / YRUN);
    if ((p[i].dim == 3 && n != 1) || p[i].q_scalar != p[0].q_scalar) return 0;
    const size_t plane = (size_t)px_of(p[i].nx) * p[i].ny * (p[i].dim == 3 ? p[i].nz : 1);
    const Layout L = layout_of(p[i]);
    total += align256(plane * rsz) * L.rplanes + align256(plane * ssz) * L.splanes;
    tilesmax += p[i].dim == 3 ? blocks3(p[i])
                              : (long long)((p[i].nx + 63) / 64) * ((p[i].ny + kTYs[0] - 1) / kTYs[0]);
    maxsites = std::max(maxsites, (size_t)sites_of(p[i]));
  }
  total += align256(sizeof(double) * 2 * (size_t)((p[0].nx * (long long)p[0].ny + 255) / 256 + 1));
  const long long padded = (tilesmax + 7) / 8 * 8;
  total += align256(sizeof(Dom) * n);
  // tile lists per tile height: "all" plus, per field, one list per group of
  // domains sharing an update factor (at most 8 groups, each padded by < 8)
  total += kNTY * (5 * (sizeof(int4) * (size_t)(padded + 64)) + 40 * 256);
  // run lists: per field, one list per group (at most 8 groups, each padded by < 8),
  // and the same runs again as per-XCD work-queue lists with their offsets
  total += 4 * (sizeof(int4) * (size_t)(runs + 128) + 8 * 256);
  total += 4 * (sizeof(int4) * (size_t)runs + 16 * 256 + 16 * 256) + align256(sizeof(WorkQ));
  total += align256(sizeof(Partial) * (size_t)tilesmax);
  total += align256(sizeof(double2) * (size_t)(runs + 1));
  total += align256(sizeof(int) * (size_t)tilesmax) + kNTY * align256(sizeof(int) * (n + 1));
  total += align256(sizeof(DiagOut) * n);
  total += align256(sizeof(unsigned long long) * n);
  total += align256(sizeof(int) * kMaxCodes);
  total += align256(sizeof(double) * maxsites * kStagePlanes);
  return total;
}

lbm_status lbm_create(const lbm_params* p, int32_t n, int32_t storage, int32_t device, void* hip_stream,
                      void* workspace, size_t workspace_bytes, lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || n < 1) return fail(nullptr, LBM_EINVAL, "no domains");
  for (int i = 0; i < n; ++i) {
    if (p[i].dim == 3 && n != 1) return fail(nullptr, LBM_EINVAL, "3D contexts hold one domain");
    if (p[i].q_scalar != p[0].q_scalar) return fail(nullptr, LBM_EINVAL, "the domains of a context share one scalar lattice");
  }
  if (storage < 0 || storage > 3) return fail(nullptr, LBM_EINVAL, "bad storage format");
  for (int i = 0; i < n; ++i) {
    const std::string m = validate(p[i], i);
    if (!m.empty()) return fail(nullptr, LBM_EINVAL, m);
  }
  {
    // the step kernels index the cycle of (up to) 4 lcm(N_chi) base steps
    // and a plane's elements in 32 bits
    long long lcm = 1;
    for (int i = 0; i < n; ++i) {
      for (int N : {p[i].N_phi, p[i].N_U, p[i].N_T, p[i].N_F}) {
        lcm = ipow_lcm(lcm, N);
        if (lcm > (1LL << 29)) return fail(nullptr, LBM_EINVAL, "the update factors' lcm exceeds 2^29");
      }
      const int esz = storage == LBM_STORE_F64 ? 8 : 4;
      const long long nz = p[i].dim == 3 ? p[i].nz : 1;
      if ((long long)px_of(p[i].nx) * p[i].ny * nz * esz >= (1LL << 32))
        return fail(nullptr, LBM_EINVAL, "domain " + std::to_string(i) + ": one field plane exceeds 4 GiB");
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, LBM_EDEVICE, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "hipSetDevice failed");

  const size_t need = lbm_workspace_bytes(p, n, storage);
  auto* c = new lbm_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->storage = storage;
  sizes_of(storage, c->rsz, c->ssz);
  switch (storage) {
    case LBM_STORE_F64: c->ops = make_ops<double, double>(); c->ops3 = make_ops3<double, double>(); break;
    case LBM_STORE_F32: c->ops = make_ops<float, float>(); c->ops3 = make_ops3<float, float>(); break;
    case LBM_STORE_F16: c->ops = make_ops<float, __half>(); c->ops3 = make_ops3<float, __half>(); break;
    default: c->ops = make_ops<float, __hip_bfloat16>(); c->ops3 = make_ops3<float, __hip_bfloat16>(); break;
  }
  c->dim = p[0].dim;
  c->ndom = n;
  c->P.assign(p, p + n);
  c->initialised.assign(n, false);
  if (workspace) {
    if (workspace_bytes < need) {
      delete c;
      return fail(nullptr, LBM_ENOMEM, "workspace smaller than lbm_workspace_bytes()");
    }
    c->ws = workspace;
    c->ws_bytes = workspace_bytes;
  } else {
    if (hipMalloc(&c->ws, need) != hipSuccess) {
      delete c;
      return fail(nullptr, LBM_ENOMEM, "hipMalloc of the workspace failed");
    }
    c->own_ws = true;
    c->ws_bytes = need;
  }
  char* cur = (char*)c->ws;
  auto take = [&](size_t bytes) {
    void* r = cur;
    cur += align256(bytes);
    return r;
  };

  // domains and their planes
  c->H.resize(n);
  long long lcm = 1;
  int rbase = 0;
  for (int i = 0; i < n; ++i) {
    const lbm_params& q = p[i];
    Dom& D = c->H[i];
    memset(&D, 0, sizeof D);
    D.nx = q.nx;
    D.ny = q.ny;
    D.nz = q.dim == 3 ? q.nz : 1;
    D.dim = q.dim;
    D.rbase = rbase;
    D.nruns = q.dim == 2 ? ((q.nx + YCOL - 1) / YCOL) * ((q.ny + YRUN - 1) / YRUN) : 0;
    rbase += D.nruns;
    D.px = px_of(q.nx);
    D.plane = (long long)D.px * q.ny * D.nz;
    for (int a = 0; a < 3; ++a) {
      D.bc[a] = q.bc[a];
      D.fbc[a] = q.flow_bc[a];
    }
    D.T_pulled = q.T_mode == LBM_T_PULLED;
    D.T_dirlow = q.T_mode == LBM_T_DIRICHLET_LOW;
    D.T_grad = q.T_grad;
    D.V_pull = q.V_pull;
    D.z_front = q.z_front;
    D.Fz = q.Fb[2];
    D.N_phi = q.N_phi;
    D.N_U = q.N_U;
    D.N_T = q.N_T;
    D.N_F = q.N_F;
    D.has_U = q.has_U;
    D.has_T = q.has_T;
    D.has_F = q.has_flow;
    D.accum = q.coupling == LBM_COUPLE_ACCUM;
    D.gradeq40 = q.grad_phi == LBM_GRAD_EQ40;
    D.T_var = (q.kappa_S != q.kappa_L) || (q.rhoCp_S != q.rhoCp_L);
    D.dt_base = q.dt_base;
    D.W0 = q.W0;
    D.tau0 = q.tau0;
    D.eps = q.eps_s;
    D.lam = q.lam;
    D.Mc = q.Mc;
    D.kc = q.k;
    D.cth = cos(q.theta_c);
    D.sth = sin(q.theta_c);
    D.D_L = q.D_L;
    D.D_S = q.D_S;
    D.C_inf = q.C_inf;
    D.kS = q.kappa_S;
    D.kL = q.kappa_L;
    D.rcS = q.rhoCp_S;
    D.rcL = q.rhoCp_L;
    D.rho_L = q.rho_L;
    D.L_h = q.L_h;
    D.T_m = q.T_m;
    D.m_L = q.m_L;
    D.Cp_L = q.Cp_L;
    D.nu = q.nu;
    D.s_e = q.s_e;
    D.s_eps = q.s_eps;
    D.s_q = q.s_q;
    D.u_in = q.u_in;
    D.Fx = q.Fb[0];
    D.Fy = q.Fb[1];
    D.U0 = q.U0;
    D.T0 = q.T0;
    D.u0_liquid = q.u0_liquid_only;
    D.qs = q.q_scalar;
    {
      double* K = D.kd;
      K[K_DTPHI] = q.N_phi * q.dt_base;
      K[K_W2T] = q.W0 * q.W0 / q.tau0;
      K[K_INVTAU0] = 1.0 / q.tau0;
      K[K_EPS] = q.eps_s;
      K[K_LAM] = q.lam;
      K[K_MC] = q.Mc;
      K[K_CTH] = cos(q.theta_c);
      K[K_STH] = sin(q.theta_c);
      K[K_INVLHCP] = q.Cp_L / q.L_h;
      K[K_THOFF] = q.T_m + q.m_L * q.C_inf;
      K[K_OMK] = 1.0 - q.k;
      K[K_OPK] = 1.0 + q.k;
      K[K_CJ] = q.W0 / (2.0 * 1.4142135623730951);
      K[K_CT] = q.rho_L * q.L_h;
      K[K_RCS] = q.rhoCp_S;
      K[K_RCL] = q.rhoCp_L;
      K[K_HRCS] = 0.5 * q.rhoCp_S;
      K[K_HRCL] = 0.5 * q.rhoCp_L;
      K[K_HKS] = 0.5 * q.kappa_S;
      K[K_HKL] = 0.5 * q.kappa_L;
      K[K_DTU] = q.N_U * q.dt_base;
      K[K_DTT] = q.N_T * q.dt_base;
      K[K_DS] = q.D_S;
      K[K_DL] = q.D_L;
      K[K_U0] = q.U0;
      K[K_T0] = q.T0;
      K[K_ALPHAL] = q.kappa_L / q.rhoCp_L;
      K[K_HDRC] = 0.5 * (q.rhoCp_S - q.rhoCp_L);
      K[K_DTF] = q.N_F * q.dt_base;
      for (int j = 0; j < K_N; ++j) D.kf[j] = (float)K[j];
    }
    const size_t pr = D.plane * c->rsz, ps = D.plane * c->ssz;
    const int d3 = q.dim == 3;
    for (int b = 0; b < 4; ++b) D.phi[b] = take(pr);
    for (int b = 0; b < 2; ++b) D.sphi[b] = take(align256(ps) * (q.q_scalar - 1));
    if (q.has_U) {
      for (int b = 0; b < 4; ++b) D.U[b] = take(pr);
      for (int b = 0; b < 2; ++b) D.jU[b] = take(align256(pr) * q.dim);   // first moment in R
      D.PU = take(pr);
    }
    if (q.has_T) {
      for (int b = 0; b < 4; ++b) D.T[b] = take(pr);
      for (int b = 0; b < 2; ++b) D.jT[b] = take(align256(ps) * q.dim);
      D.PT = take(pr);
    }
    if (q.has_flow) {
      for (int b = 0; b < 2; ++b) {
        D.rho[b] = take(pr);
        D.sF[b] = take(align256(ps) * (d3 ? 18 : 8));
        D.vel[b] = take(align256(pr) * q.dim);
      }
    }
    if (D.gradeq40)
      for (int b = 0; b < 2; ++b) D.gq[b] = take(align256(pr) * 3);
    lcm = ipow_lcm(lcm, q.N_phi);
    if (q.has_U) lcm = ipow_lcm(lcm, q.N_U);
    if (q.has_T) lcm = ipow_lcm(lcm, q.N_T);
    if (q.has_flow) lcm = ipow_lcm(lcm, q.N_F);
  }
  c->qs = p[0].q_scalar;
  c->fusable = true;
  for (int i = 0; i < n; ++i) c->fusable &= p[i].dim == 2 && p[i].q_scalar == 5 && p[i].nx >= 8 && p[i].ny >= 8;
  c->deferrable = p[0].dim == 2 && p[0].q_scalar == 5;
  for (int i = 0; i < n; ++i)
    c->deferrable &= p[i].N_phi == 1 && p[i].coupling == LBM_COUPLE_INSTANT && p[i].nx >= 8 && p[i].ny >= 8;
  c->marchable = true;
  for (int i = 0; i < n; ++i) c->marchable &= p[i].dim == 2 && p[i].nx >= 16 && p[i].ny >= 16;
  // the Eq. (40) phase gradient exists in the tiled phase kernel only
  for (int i = 0; i < n; ++i)
    if (p[i].grad_phi == LBM_GRAD_EQ40) c->marchable = c->fusable = c->deferrable = false;
  {
    long long runs = 0;   // a column run is one block: marching pays when they are many
    for (int i = 0; i < n; ++i) runs += (long long)((p[i].nx + YCOL - 1) / YCOL) * ((p[i].ny + YRUN - 1) / YRUN);
    c->march_big = runs >= 4 * 256;
    c->march_pick = c->march_big;
  }
  // the buffer indices of phi, U and T (write counts mod 4) repeat too;
  // the counts are even over 2 lcm, so doubling once makes them multiples of 4
  c->cycle = 2 * lcm;
  for (int i = 0; i < n; ++i) {
    const bool inst = p[i].coupling == LBM_COUPLE_INSTANT;
    const long long wphi = c->cycle / p[i].N_phi;
    const long long wU = p[i].has_U ? (inst ? wphi : 0) + c->cycle / p[i].N_U : 0;
    const long long wT = p[i].has_T ? (inst && p[i].T_mode != LBM_T_PULLED ? wphi : 0) + c->cycle / p[i].N_T : 0;
    if (wphi % 4 != 0 || wU % 4 != 0 || wT % 4 != 0) {
      c->cycle *= 2;
      break;
    }
  }
  c->d_dom = (Dom*)take(sizeof(Dom) * n);

  // tile lists (three tile heights), groups by update factor
  long long tilesmax = 0;
  size_t maxsites = 0;
  for (int i = 0; i < n; ++i) {
    tilesmax += p[i].dim == 3 ? blocks3(p[i])
                              : (long long)((p[i].nx + 63) / 64) * ((p[i].ny + kTYs[0] - 1) / kTYs[0]);
    maxsites = std::max(maxsites, (size_t)sites_of(p[i]));
  }
  if (c->dim == 3) {
    c->nblk3 = (int)blocks3(p[0]);
    c->nfront = (int)((p[0].nx * (long long)p[0].ny + 255) / 256);
    c->s.front = (double*)take(sizeof(double) * 2 * (c->nfront + 1));
  }
  auto build = [&](const std::vector<int>& doms, int ti, TileSet& ts, std::vector<int>* slot0) -> lbm_status {
    const int TY = kTYs[ti];
    std::vector<int4> sp;
    // slots are the spatial index over all domains, so every list writes the
    // same partial slot for a given tile
    std::vector<int> base(n + 1, 0);
    for (int i = 0; i < n; ++i)
      base[i + 1] = base[i] + ((p[i].nx + 63) / 64) * ((p[i].ny + TY - 1) / TY);
    for (int d : doms) {
      const int ntx = (p[d].nx + 63) / 64, nty = (p[d].ny + TY - 1) / TY;
      for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) sp.push_back(make_int4(d, tx * 64, ty * TY, base[d] + ty * ntx + tx));
    }
    if (slot0) *slot0 = base;
    std::vector<int4> o = xcd_order(sp);
    ts.d = (int4*)take(sizeof(int4) * o.size());
    ts.n = (int)o.size();
    HIPCHK(c, hipMemcpy(ts.d, o.data(), sizeof(int4) * o.size(), hipMemcpyHostToDevice));
    return LBM_OK;
  };
  std::vector<int> alld(n);
  std::iota(alld.begin(), alld.end(), 0);
  std::vector<int> slot0[kNTY];
  for (int ti = 0; ti < kNTY; ++ti) {
    if (c->dim == 3) {
      slot0[ti] = {0, c->nblk3};   // 3D: one partial slot per block of 256 sites
      continue;
    }
    lbm_status s = build(alld, ti, c->all[ti], &slot0[ti]);
    if (s != LBM_OK) {
      lbm_destroy(c);
      return fail(nullptr, s, g_create_error.empty() ? "tile upload failed" : g_create_error);
    }
  }
  auto make_groups = [&](int field, std::vector<Group>& gs) -> lbm_status {
    std::map<int, std::vector<int>> by;
    for (int i = 0; i < n; ++i) {
      const lbm_params& q = p[i];
      if (field == 0) by[q.N_phi].push_back(i);
      if (field == 1 && q.has_U) by[q.N_U].push_back(i);
      if (field == 2 && q.has_T) by[q.N_T].push_back(i);
      if (field == 3 && q.has_flow) by[q.N_F].push_back(i);
    }
    if (by.size() > 1 && (int)by.size() > 8) return LBM_EINVAL;
    for (auto& kv : by) {
      Group g;
      g.N = kv.first;
      if (c->dim == 3) {   // 3D kernels take the whole domain, no tile lists
        gs.push_back(g);
        continue;
      }
      for (int ti = 0; ti < kNTY; ++ti) {
        if (by.size() == 1 && (int)kv.second.size() == n) {
          g.ts[ti] = c->all[ti];
        } else {
          lbm_status s = build(kv.second, ti, g.ts[ti], nullptr);
          if (s != LBM_OK) return s;
        }
      }
      {
        std::vector<int4> sp;
        for (int d : kv.second)
          for (int y0 = 0; y0 < p[d].ny; y0 += YRUN)
            for (int x0 = 0; x0 < p[d].nx; x0 += YCOL) sp.push_back(make_int4(d, x0, y0, std::min(p[d].ny, y0 + YRUN)));
        std::vector<int4> o = xcd_order(sp);
        g.runs.d = (int4*)take(sizeof(int4) * o.size());
        g.runs.n = (int)o.size();
        HIPCHK(c, hipMemcpy(g.runs.d, o.data(), sizeof(int4) * o.size(), hipMemcpyHostToDevice));
      }
      if (field == 0) {   // the marching phase kernel: runs 64 wide
        std::vector<int4> sp;
        for (int d : kv.second)
          for (int y0 = 0; y0 < p[d].ny; y0 += YRUN)
            for (int x0 = 0; x0 < p[d].nx; x0 += 64) sp.push_back(make_int4(d, x0, y0, std::min(p[d].ny, y0 + YRUN)));
        std::vector<int4> o = xcd_order(sp);
        g.runs64.d = (int4*)take(sizeof(int4) * o.size());
        g.runs64.n = (int)o.size();
        HIPCHK(c, hipMemcpy(g.runs64.d, o.data(), sizeof(int4) * o.size(), hipMemcpyHostToDevice));
      }
      // work-queue lists: the domains by decreasing size (ties keep their
      // order), each domain's runs row by row, cut into eight contiguous
      // lists of equal length (a domain is split only at the cuts)
      auto make_q = [&](int width, QList& ql) -> lbm_status {
        std::vector<int> order = kv.second;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sites_of(p[a]) > sites_of(p[b]); });
        std::vector<int4> all;
        for (int d : order)
          for (int y0 = 0; y0 < p[d].ny; y0 += YRUN)
            for (int x0 = 0; x0 < p[d].nx; x0 += width)
              all.push_back(make_int4(d, x0, y0, std::min(p[d].ny, y0 + YRUN)));
        int off[9];
        for (int x = 0; x <= 8; ++x) off[x] = (int)((long long)all.size() * x / 8);
        int4* items = (int4*)take(sizeof(int4) * std::max<size_t>(all.size(), 1));
        int* qoff = (int*)take(sizeof(int) * 9);
        HIPCHK(c, hipMemcpy(items, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(qoff, off, sizeof(int) * 9, hipMemcpyHostToDevice));
        ql = QList{items, qoff, (int)all.size()};
        return LBM_OK;
      };
      {
        lbm_status s = make_q(YCOL, g.q);
        if (s == LBM_OK && field == 0) s = make_q(64, g.q64);
        if (s != LBM_OK) return s;
      }
      gs.push_back(g);
    }
    return LBM_OK;
  };
  // at most one extra list per field beyond "all": keep the workspace bound
  for (int f = 0; f < 4; ++f) {
    std::vector<Group>& gs = f == 0 ? c->g_phi : f == 1 ? c->g_U : f == 2 ? c->g_T : c->g_F;
    lbm_status s = make_groups(f, gs);
    if (s != LBM_OK) {
      lbm_destroy(c);
      return fail(nullptr, LBM_EINVAL, "too many distinct update factors for one field (max 8)");
    }
  }
  c->one_U = c->g_U.size() == 1;
  c->one_T = c->g_T.size() == 1 && c->g_phi.size() == 1;
  for (int i = 0; i < n; ++i) {
    c->one_U &= p[i].has_U != 0;
    c->one_T &= p[i].has_T != 0 && p[i].T_mode != LBM_T_PULLED && p[i].coupling == LBM_COUPLE_INSTANT;
  }
  c->s.part = (Partial*)take(sizeof(Partial) * (size_t)tilesmax);
  c->s.rmax = (double2*)take(sizeof(double2) * (size_t)(rbase + 1));
  c->d_wq = (WorkQ*)take(sizeof(WorkQ));
  if (hipMemset(c->d_wq, 0, sizeof(WorkQ)) != hipSuccess) {
    lbm_destroy(c);
    return fail(nullptr, LBM_EDEVICE, "clearing the work queues failed");
  }
  if (hipMemset(c->s.rmax, 0, sizeof(double2) * (size_t)(rbase + 1)) != hipSuccess) {
    lbm_destroy(c);
    return fail(nullptr, LBM_EDEVICE, "clearing the run maxima failed");
  }
  c->d_slot = (int*)take(sizeof(int) * (size_t)tilesmax);
  for (int ti = 0; ti < kNTY; ++ti) c->d_slot0[ti] = (int*)take(sizeof(int) * (n + 1));
  c->s.diag = (DiagOut*)take(sizeof(DiagOut) * n);
  c->ws_s = c->s;
  c->nparts = tilesmax;
  c->nrmax = rbase + 1;
  c->scratch_bytes = align256(sizeof(Partial) * (size_t)tilesmax) + align256(sizeof(double2) * (size_t)(rbase + 1)) +
                     align256(sizeof(DiagOut) * n) + align256(sizeof(double) * 2 * (size_t)(c->nfront + 1));
  c->h_d.resize(n);
  if (hipHostMalloc((void**)&c->h_diag, sizeof(DiagOut) * n) != hipSuccess ||
      hipHostMalloc((void**)&c->h_first, sizeof(unsigned long long) * n) != hipSuccess ||
      hipHostMalloc((void**)&c->h_front, sizeof(double) * (2 * (size_t)c->nfront + 2)) != hipSuccess) {
    lbm_destroy(c);
    return fail(nullptr, LBM_ENOMEM, "pinned host staging allocation failed");
  }
  c->d_first = (unsigned long long*)take(sizeof(unsigned long long) * n);
  c->d_codes = (int*)take(sizeof(int) * kMaxCodes);
  c->m0.assign(n, 0.0);
  {
    long long rows = 0;   // the screen's blocks walk rows of the tallest domain, four per block
    for (int i = 0; i < n; ++i) rows = std::max(rows, (long long)p[i].ny * (p[i].dim == 3 ? p[i].nz : 1));
    c->nf_blocks = (int)std::max(1LL, std::min((rows + 3) / 4, n == 1 ? 2048LL : 64LL));
  }
  c->stage_elems = maxsites * kStagePlanes;
  c->d_stage = (double*)take(sizeof(double) * c->stage_elems);
  if ((size_t)(cur - (char*)c->ws) > c->ws_bytes) {
    lbm_destroy(c);
    return fail(nullptr, LBM_ENOMEM, "internal: workspace layout overflow");
  }
  {
    std::vector<int> slots((size_t)tilesmax);
    std::iota(slots.begin(), slots.end(), 0);
    if (hipMemcpy(c->d_slot, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice) != hipSuccess) {
      lbm_destroy(c);
      return fail(nullptr, LBM_EDEVICE, "slot upload failed");
    }
    for (int ti = 0; ti < kNTY; ++ti)
      if (hipMemcpy(c->d_slot0[ti], slot0[ti].data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice) != hipSuccess) {
        lbm_destroy(c);
        return fail(nullptr, LBM_EDEVICE, "slot upload failed");
      }
    if (hipMemset(c->d_first, 0xff, sizeof(unsigned long long) * n) != hipSuccess ||
        hipMemset(c->s.part, 0, sizeof(Partial) * (size_t)tilesmax) != hipSuccess) {
      lbm_destroy(c);
      return fail(nullptr, LBM_EDEVICE, "partial clear failed");
    }
  }
  static_scratch_setup(device);   // the allocation-free entry point's scratch on this device
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    lbm_destroy(c);
    return fail(nullptr, LBM_EDEVICE, "stream creation failed");
  }
  if (upload_doms(c) != LBM_OK) {
    std::string m = c->err;
    lbm_destroy(c);
    return fail(nullptr, LBM_EDEVICE, m);
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_init_seeds(lbm_ctx* c, int32_t dom, int32_t n_seeds, const double* centres, const double* radii) {
  if (!c) return LBM_EINVAL;
  if (dom < 0 || dom >= c->ndom) return fail(c, LBM_EINVAL, "bad domain index");
  if (n_seeds < 0 || n_seeds > MAX_SEEDS) return fail(c, LBM_EINVAL, "0..4 seeds per domain");
  if (n_seeds > 0 && (!centres || !radii)) return fail(c, LBM_EINVAL, "NULL seed arrays");
  if (c->dim == 3) return fail(c, LBM_EINVAL, "3D domains are initialised with lbm_init_front");
  HIPCHK(c, hipSetDevice(c->device));
  Dom& D = c->H[dom];
  D.nseeds = n_seeds;
  for (int s = 0; s < n_seeds; ++s) {
    D.seed[s][0] = centres[2 * s];
    D.seed[s][1] = centres[2 * s + 1];
    D.seed[s][2] = radii[s];
  }
  lbm_status st = upload_doms(c);
  if (st != LBM_OK) return st;
  c->ops.init(c->stream, c->d_dom, dom, (long long)D.nx * D.ny, nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemsetAsync(c->d_first + dom, 0xff, sizeof(unsigned long long), c->stream));
  c->initialised[dom] = true;
  c->need_m0 = true;
  c->k = 0;
  return LBM_OK;
}

lbm_status lbm_init_front(lbm_ctx* c, int32_t dom, const double* xi) {
  if (!c) return LBM_EINVAL;
  if (dom < 0 || dom >= c->ndom) return fail(c, LBM_EINVAL, "bad domain index");
  HIPCHK(c, hipSetDevice(c->device));
  Dom& D = c->H[dom];
  const double* dxi = nullptr;
  const size_t ncol = c->dim == 3 ? (size_t)D.nx * D.ny : (size_t)D.nx;
  if (xi) {
    HIPCHK(c, hipMemcpyAsync(c->d_stage, xi, sizeof(double) * ncol, hipMemcpyHostToDevice, c->stream));
    dxi = c->d_stage;
  }
  if (c->dim == 3) {
    c->ops3.init(D, c->stream, c->d_dom, dxi);
    c->ops3.set_koff(c->stream, c->d_dom, 0);
    c->koff = 0;
  } else {
    D.nseeds = 0;   // no seed tips for a front
    lbm_status st = upload_doms(c);
    if (st != LBM_OK) return st;
    c->ops.init(c->stream, c->d_dom, dom, (long long)D.nx * D.ny, dxi);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemsetAsync(c->d_first + dom, 0xff, sizeof(unsigned long long), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->initialised[dom] = true;
  c->need_m0 = true;
  c->k = 0;
  return LBM_OK;
}

lbm_status lbm_configure(lbm_ctx* c, int32_t tile_rows, int32_t flags) {
  if (!c) return LBM_EINVAL;
  if (c->dim == 3) {   // 3D: rows of the stencil kernels' 64-wide tiles
    if (tile_rows != 0 && tile_rows != 4 && tile_rows != 8)
      return fail(c, LBM_EINVAL, "3D tile_rows must be 0, 4 or 8");
    if (tile_rows != c->rows3) {
      // fewer blocks at other heights: the transfer and U partials of the
      // blocks that no longer exist must not linger in the reductions
      HIPCHK(c, hipStreamSynchronize(c->stream));
      HIPCHK(c, hipMemset(c->ws_s.part, 0, sizeof(Partial) * (size_t)c->nparts));
    }
    c->rows3 = tile_rows;
    // 0: the autotuner picks each kernel's height and z runs at the next
    // step; a fixed height keeps the z runs picked so far (or the defaults)
    c->autotune = tile_rows == 0;
    if (tile_rows == 0) c->tuned = false;
  } else if (tile_rows == 0) {
    c->autotune = true;
    c->tuned = false;
  } else {
    int ti = -1;
    for (int i = 0; i < kNTY; ++i)
      if (kTYs[i] == tile_rows) ti = i;
    if (ti < 0) return fail(c, LBM_EINVAL, "tile_rows must be 0, 4, 8, 16 or 32");
    c->ty_index = ti;
    c->autotune = false;
    c->tuned = true;
  }
  if (flags & ~127) return fail(c, LBM_EINVAL, "unknown configure flags");
  if ((flags & LBM_CFG_MARCH) && (flags & LBM_CFG_TILES))
    return fail(c, LBM_EINVAL, "LBM_CFG_MARCH and LBM_CFG_TILES exclude each other");
  if ((flags & LBM_CFG_QUEUE) && (flags & LBM_CFG_GRID))
    return fail(c, LBM_EINVAL, "LBM_CFG_QUEUE and LBM_CFG_GRID exclude each other");
  c->use_graph = (flags & LBM_CFG_GRAPH) != 0;
  c->fuse = (flags & LBM_CFG_FUSE_TRANSFER) != 0;
  c->march = (flags & LBM_CFG_MARCH) ? 1 : (flags & LBM_CFG_TILES) ? -1 : 0;
  c->defer = (flags & LBM_CFG_NO_DEFER) == 0;
  c->queue = (flags & LBM_CFG_QUEUE) ? 1 : (flags & LBM_CFG_GRID) ? -1 : 0;
  if (c->queue != 0) c->use_q = c->queue > 0;
  if (c->gexec) {   // the captured cycle follows the kernel choice
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  return LBM_OK;
}

int64_t lbm_steps_done(const lbm_ctx* c) { return c ? c->k : -1; }

int32_t lbm_marching(const lbm_ctx* c) { return c ? (use_march(c) ? 1 : 0) : -1; }

int32_t lbm_tile_rows(const lbm_ctx* c) {
  if (!c) return -1;
  if (c->dim == 3) return c->rows3;
  if (c->autotune && !c->tuned) return 0;
  return kTYs[c->ty_index];
}

lbm_status lbm_kernel_times(lbm_ctx* c, int32_t reps, double* ms_out, double* per_step) {
  if (!c || !ms_out || reps < 1) return c ? fail(c, LBM_EINVAL, "bad arguments") : LBM_EINVAL;
  for (int d = 0; d < c->ndom; ++d)
    if (!c->initialised[d]) return fail(c, LBM_ESTATE, "lbm_init_seeds has not been called for every domain");
  HIPCHK(c, hipSetDevice(c->device));
  if (c->autotune && !c->tuned) {
    lbm_status s = c->dim == 3 ? autotune3(c) : autotune(c);
    if (s != LBM_OK) return s;
  }
  const int ti = c->ty_index, TY = kTYs[ti];
  const bool fused = c->dim == 2 && c->fuse && c->fusable;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  auto due = [&](int N) { return (c->k / N + 1) * (long long)N; };
  for (int kind = 0; kind < 5; ++kind) {
    const std::vector<Group>& gs = kind <= 1 ? c->g_phi : kind == 2 ? c->g_U : kind == 3 ? c->g_T : c->g_F;
    if (gs.empty() || (kind == 1 && fused)) {   // fused: the transfer runs inside the phase kernel
      ms_out[kind] = -1.0;
      if (per_step) per_step[kind] = 0.0;
      continue;
    }
    // each group of domains sharing an update factor is timed on its own:
    // ms_out is one launch over every domain, per_step the fraction of it
    // spent per base step (groups weighted by how often they are due)
    double all = 0.0, weighted = 0.0;
    for (auto& g : gs) {
      const unsigned k = cycle_step(c, due(g.N));
      const dim3 grid(g.ts[ti].n);
      auto launch = [&]() {
        if (c->dim == 3) {
          const Dom& h = c->H[0];
          if (kind == 0) c->ops3.phase(h, c->stream, c->d_dom, k, rows3(c, 0), zblk3(c, 0));
          if (kind == 1) c->ops3.transfer(h, c->stream, c->d_dom, k, c->s.part, rows3(c, 1), zblk3(c, 1));
          if (kind == 2) c->ops3.scalar(0, h, c->stream, c->d_dom, k, c->s.part, rows3(c, 2), zblk3(c, 2));
          if (kind == 3) c->ops3.scalar(1, h, c->stream, c->d_dom, k, c->s.part, rows3(c, 3), zblk3(c, 3));
          if (kind == 4) c->ops3.flow(h, c->stream, c->d_dom, k, rows3(c, 4), zblk3(c, 4));
          return;
        }
        if (kind == 0 && fused) {
          const int tf = ty_slot(c->ops.phase_tr_rows(TY));
          c->ops.phase_tr(kTYs[tf], dim3(g.ts[tf].n), c->stream, c->d_dom, g.ts[tf].d, k, c->s.part);
        }
        if (kind == 0 && !fused && use_march(c) && c->use_q)
          c->ops.phase_ymq(c->qs, g.q64, c->d_wq, c->stream, c->d_dom, k);
        else if (kind == 0 && !fused && use_march(c))
          c->ops.phase_ym(c->qs, dim3(g.runs64.n), c->stream, c->d_dom, g.runs64.d, k);
        else if (kind == 0 && !fused)
          c->ops.phase(TY, c->qs, grid, c->stream, c->d_dom, g.ts[ti].d, k);
        if (kind == 1 && use_march(c) && c->use_q)
          c->ops.transfer_ymq(g.q, c->d_wq, c->stream, c->d_dom, k, c->s.rmax);
        else if (kind == 1 && use_march(c))
          c->ops.transfer_ym(dim3(g.runs.n), c->stream, c->d_dom, g.runs.d, k, c->s.rmax);
        else if (kind == 1)
          c->ops.transfer(TY, grid, c->stream, c->d_dom, g.ts[ti].d, k, c->s.part);
        if ((kind == 2 || kind == 3) && use_march(c) && c->use_q)
          c->ops.scalar_ymq(kind - 2, c->qs, g.q, c->d_wq, c->stream, c->d_dom, k, c->s.rmax);
        else if ((kind == 2 || kind == 3) && use_march(c))
          c->ops.scalar_ym(kind - 2, c->qs, dim3(g.runs.n), c->stream, c->d_dom, g.runs.d, k, c->s.rmax);
        else if (kind == 2 || kind == 3)
          c->ops.scalar(kind - 2, TY, c->qs, grid, c->stream, c->d_dom, g.ts[ti].d, k, c->s.part);
        if (kind == 4) c->ops.flow(TY, grid, c->stream, c->d_dom, g.ts[ti].d, k);
      };
      launch();
      HIPCHK(c, hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps; ++r) launch();
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      const double per_launch = double(ms) / reps;
      all += per_launch;
      weighted += per_launch / g.N;
    }
    ms_out[kind] = all;
    if (per_step) per_step[kind] = weighted / all;
  }
  // deferred transfers: the phase kernel with the previous step's transfer
  // runs instead of the plain one on the steps after a deferral, and the U
  // transport with its step's transfer instead of the plain one
  auto time_launch = [&](auto launch, double& out) -> lbm_status {
    launch();
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) launch();
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    out = double(ms) / reps;
    return LBM_OK;
  };
  ms_out[5] = ms_out[6] = ms_out[7] = -1.0;
  if (per_step) per_step[5] = per_step[6] = per_step[7] = 0.0;
  if (c->dim == 2 && !fused) {
    long long ndef = 0, nfu = 0;
    for (long long kk = 1; kk <= c->cycle; ++kk) {
      ndef += kk < c->cycle && defers(c, (unsigned)kk);
      nfu += fuses_U(c, (unsigned)kk);
    }
    if (ndef > 0) {
      const double fdef = double(ndef) / double(c->cycle);
      if (per_step) {
        per_step[0] *= 1.0 - fdef;
        per_step[1] *= 1.0 - fdef;
        per_step[5] = fdef;
      }
      const Group& g = c->g_phi[0];
      lbm_status s = time_launch(
          [&]() { c->ops.dtr_phase(TY, dim3(g.ts[ti].n), c->stream, c->d_dom, g.ts[ti].d, 2u, c->s.part); },
          ms_out[5]);
      if (s != LBM_OK) return s;
    }
    if (nfu > 0) {   // (every phase step is due: N_phi = 1)
      if (per_step) {
        per_step[1] -= double(nfu) / double(c->cycle);
        per_step[2] = 0.0;
        per_step[6] = double(nfu) / double(c->cycle);
      }
      const Group& g = c->g_U[0];
      const unsigned k = cycle_step(c, due(g.N));
      lbm_status s = time_launch(
          [&]() { c->ops.dtr_scalar(TY, dim3(g.ts[ti].n), c->stream, c->d_dom, g.ts[ti].d, k, c->s.part); },
          ms_out[6]);
      if (s != LBM_OK) return s;
    }
    long long ntr = 0;
    for (long long kk = 1; kk <= c->cycle; ++kk) ntr += fuses_T(c, (unsigned)kk);
    if (ntr > 0) {   // the marching transfer inside the T transport
      const double f = double(ntr) / double(c->cycle);
      if (per_step) {
        per_step[1] -= f;
        per_step[3] -= f;
        per_step[7] = f;
      }
      const Group& g = c->g_T[0];
      const unsigned k = cycle_step(c, due(std::lcm(g.N, c->g_phi[0].N)));
      lbm_status s = time_launch(
          [&]() {
            if (c->use_q) c->ops.tr_scalar_ymq(c->qs, g.q, c->d_wq, c->stream, c->d_dom, k, c->s.rmax);
            else c->ops.tr_scalar_ym(c->qs, dim3(g.runs.n), c->stream, c->d_dom, g.runs.d, k, c->s.rmax);
          },
          ms_out[7]);
      if (s != LBM_OK) return s;
    }
  }
  HIPCHK(c, hipEventDestroy(e0));
  HIPCHK(c, hipEventDestroy(e1));
  HIPCHK(c, hipGetLastError());
  for (int d = 0; d < c->ndom; ++d) c->initialised[d] = false;
  return LBM_OK;
}

// source of S_phi and J_U for the final reduction (see k_diag_final)
static int diag_src(const lbm_ctx* c) {
  return c->dim == 2 ? (c->tr_march ? 1 : 0) | (c->u_march ? 2 : 0) : 0;
}

// Reduce the diagnostics of every domain into out[0..ndom-1] (synchronises).
// Does not judge finiteness: the caller does.  Uses the host staging held
// by the context (no allocation).
static lbm_status run_diag(lbm_ctx* c, lbm_diag* out) {
  const int ti = c->ty_index, TY = kTYs[ti];
  if (c->dim == 3) {
    c->ops3.diag(c->H[0], c->stream, c->d_dom, c->k, c->s.part, c->s.front);
    diag_final(c->ndom, c->stream, c->d_dom, c->s.part, c->d_slot, c->d_slot0[ti], c->s.rmax, diag_src(c),
               c->s.diag);
    HIPCHK(c, hipMemcpyAsync(c->h_front, c->s.front, sizeof(double) * 2 * (size_t)c->nfront,
                             hipMemcpyDeviceToHost, c->stream));
  } else {
    c->ops.diag_tiles(TY, dim3(c->all[ti].n), c->stream, c->d_dom, c->all[ti].d, c->k, c->s.part);
    diag_final(c->ndom, c->stream, c->d_dom, c->s.part, c->d_slot, c->d_slot0[ti], c->s.rmax, diag_src(c),
               c->s.diag);
    c->ops.tips(c->ndom, c->stream, c->d_dom, c->k, c->s.diag);
  }
  HIPCHK(c, hipGetLastError());
  DiagOut* h = c->h_diag;
  unsigned long long* first = c->h_first;
  HIPCHK(c, hipMemcpyAsync(h, c->s.diag, sizeof(DiagOut) * c->ndom, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(first, c->d_first, sizeof(unsigned long long) * c->ndom, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->dim == 3) {
    double m = -1e300, sm = 0.0;
    for (int b = 0; b < c->nfront; ++b) {
      m = std::max(m, c->h_front[2 * b]);
      sm += c->h_front[2 * b + 1];
    }
    for (int j = 0; j < 16; ++j) h[0].tip[j] = 0.0;
    h[0].tip[0] = m;
    h[0].tip[1] = sm / (double(c->H[0].nx) * c->H[0].ny);
  }
  for (int d = 0; d < c->ndom; ++d) {
    lbm_diag& o = out[d];
    memset(&o, 0, sizeof o);
    o.step = c->k;
    o.solid = h[d].solid;
    o.M_C = h[d].M_C;
    o.enthalpy = h[d].enthalpy;
    o.mass = h[d].mass;
    o.S_phi = h[d].S_phi;
    o.J_U = h[d].J_U;
    for (int j = 0; j < 16; ++j) o.tip[j] = h[d].tip[j];
    o.nonfinite = h[d].nonfinite;
    o.t = double(c->k) * c->P[d].dt_base;
    o.R_M = c->m0[d] != 0.0 ? (h[d].M_C - c->m0[d]) / c->m0[d] : 0.0;
    o.first_nonfinite_step = first[d] == ~0ULL ? -1 : (int64_t)first[d];
  }
  return LBM_OK;
}

// Screen the macroscopic planes of every domain after the current step
// (absolute step c->k) for non-finite values; the device keeps the first
// step at which each domain failed a screen.
static void screen(lbm_ctx* c) {
  nonfinite_check(c->storage == LBM_STORE_F64, c->ndom, c->nf_blocks, c->stream, c->d_dom, c->k, c->d_first);
}

// The body of both stepping entry points.  With use_static the scratch is
// the device's static array (already selected in c->s), no graph is
// captured or replayed and the autotuner does not run.
static lbm_status step_impl(lbm_ctx* c, int64_t n, lbm_diag* diag, bool use_static) {
  if (c->need_m0) {   // M_C(0) of every domain, for R_M
    lbm_status s = run_diag(c, c->h_d.data());
    if (s != LBM_OK) return s;
    for (int d = 0; d < c->ndom; ++d) c->m0[d] = c->h_d[d].M_C;
    c->need_m0 = false;
  }
  if (!use_static && c->autotune && !c->tuned) {
    lbm_status s = c->dim == 3 ? autotune3(c) : autotune(c);
    if (s != LBM_OK) return s;
  }
  long long left = n;
  bool screened = true;
  while (left > 0) {
    const bool graphable = !use_static && c->use_graph && c->cycle <= kMaxGraphSteps;
    if (graphable && c->k % c->cycle == 0 && left >= c->cycle) {
      if (!c->gexec || c->graph_ty != c->ty_index) {
        if (c->gexec) {
          HIPCHK(c, hipGraphExecDestroy(c->gexec));
          c->gexec = nullptr;
        }
        hipGraph_t g;
        HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        for (long long j = 1; j <= c->cycle; ++j) launch_step(c, c->cap_stream, (unsigned)j);
        HIPCHK(c, hipStreamEndCapture(c->cap_stream, &g));
        hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(c, LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        c->graph_ty = c->ty_index;
      }
      if (c->dim == 3 && c->koff != c->k) {   // absolute step for the time-dependent 3D walls
        c->ops3.set_koff(c->stream, c->d_dom, c->k);
        c->koff = c->k;
      }
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      c->k += c->cycle;
      left -= c->cycle;
      screen(c);   // once per replayed cycle
      screened = true;
    } else {
      const long long base = c->k - c->k % c->cycle;
      if (c->dim == 3 && c->koff != base) {
        c->ops3.set_koff(c->stream, c->d_dom, base);
        c->koff = base;
      }
      launch_step(c, c->stream, cycle_step(c, c->k + 1), left == 1);
      c->k += 1;
      left -= 1;
      screened = false;
      if (c->k % c->cycle == 0 && left > 0) {   // direct launches: screen at every cycle end too
        screen(c);
        screened = true;
      }
    }
  }
  if (!screened) screen(c);
  HIPCHK(c, hipGetLastError());
  const bool want = diag != nullptr;
  if (!want) {
    diag = c->h_d.data();
    HIPCHK(c, hipMemcpyAsync(c->h_first, c->d_first, sizeof(unsigned long long) * c->ndom,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int d = 0; d < c->ndom; ++d) {
      diag[d].nonfinite = 0;
      diag[d].first_nonfinite_step = c->h_first[d] == ~0ULL ? -1 : (int64_t)c->h_first[d];
    }
  } else {
    lbm_status s = run_diag(c, diag);
    if (s != LBM_OK) return s;
  }
  for (int d = 0; d < c->ndom; ++d)
    if (diag[d].first_nonfinite_step >= 0 || diag[d].nonfinite > 0) {
      char b[160];
      snprintf(b, sizeof b, "non-finite values in domain %d (first found after base step %lld)", d,
               (long long)diag[d].first_nonfinite_step);
      return fail(c, LBM_EUNSTABLE, b);
    }
  return LBM_OK;
}

lbm_status lbm_step_multirate(lbm_ctx* c, int64_t n, lbm_diag* diag) {
  if (!c) return LBM_EINVAL;
  if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
  for (int d = 0; d < c->ndom; ++d)
    if (!c->initialised[d]) return fail(c, LBM_ESTATE, "lbm_init_seeds has not been called for every domain");
  HIPCHK(c, hipSetDevice(c->device));
  return step_impl(c, n, diag, false);
}

lbm_status lbm_step_multirate_static(lbm_ctx* c, int64_t n, lbm_diag* diag) {
  if (!c) return LBM_EINVAL;
  if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
  if (c->scratch_bytes > kScratchBytes) {
    char b[200];
    snprintf(b, sizeof b, "this context needs %zu bytes of reduction scratch; the static scratch holds %zu",
             c->scratch_bytes, kScratchBytes);
    return fail(c, LBM_EINVAL, b);
  }
  for (int d = 0; d < c->ndom; ++d)
    if (!c->initialised[d]) return fail(c, LBM_ESTATE, "lbm_init_seeds has not been called for every domain");
  HIPCHK(c, hipSetDevice(c->device));
  void* base = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
  if (!base) {
    const hipError_t e = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_err[c->device] : hipErrorInvalidDevice;
    return fail(c, LBM_EDEVICE, std::string("static scratch address unavailable: ") + hipGetErrorString(e));
  }
  char* cur = (char*)base;
  auto take = [&](size_t bytes) {
    void* r = cur;
    cur += align256(bytes);
    return r;
  };
  Scratch st;
  st.part = (Partial*)take(sizeof(Partial) * (size_t)c->nparts);
  st.rmax = (double2*)take(sizeof(double2) * (size_t)c->nrmax);
  st.diag = (DiagOut*)take(sizeof(DiagOut) * c->ndom);
  st.front = (double*)take(sizeof(double) * 2 * (size_t)(c->nfront + 1));
  // the array keeps the previous call's contents (possibly another
  // context's): start from zero partials and run maxima, with a kernel
  const long long words = (long long)(((char*)st.diag - (char*)st.part) / sizeof(unsigned long long));
  k_zero_words<<<(unsigned)std::min<long long>((words + 255) / 256, 1024), 256, 0, c->stream>>>(
      (unsigned long long*)st.part, words);
  HIPCHK(c, hipGetLastError());
  c->s = st;
  const lbm_status r = step_impl(c, n, diag, true);
  c->s = c->ws_s;
  return r;
}

static int codes_for(const Dom& D, uint32_t mask, int* codes) {
  int n = 0;
  if (D.dim == 3) {
    if (mask & LBM_F_PHI) codes[n++] = 0;
    if (mask & LBM_F_U) codes[n++] = 1;
    if (mask & LBM_F_T) codes[n++] = 2;
    if (mask & LBM_F_RHO) codes[n++] = 3;
    if (mask & LBM_F_VEL) for (int a = 0; a < 3; ++a) codes[n++] = 4 + a;
    if (mask & LBM_F_POP_PHI) for (int q = 0; q < 7; ++q) codes[n++] = 10 + q;
    if (mask & LBM_F_JU) for (int a = 0; a < 3; ++a) codes[n++] = 20 + a;
    if (mask & LBM_F_JT) for (int a = 0; a < 3; ++a) codes[n++] = 30 + a;
    if (mask & LBM_F_POP_F) for (int q = 0; q < 19; ++q) codes[n++] = 40 + q;
    if (mask & LBM_F_PEND_U) codes[n++] = 90;
    if (mask & LBM_F_PEND_T) codes[n++] = 91;
    if (mask & LBM_F_SPHI) for (int q = 0; q < 6; ++q) codes[n++] = 60 + q;
    if (mask & LBM_F_SF) for (int q = 0; q < 18; ++q) codes[n++] = 70 + q;
    if (mask & LBM_F_SU) codes[n++] = 8;
    if (mask & LBM_F_ST) codes[n++] = 9;
    return n;
  }
  if (mask & LBM_F_PHI) codes[n++] = 0;
  if (mask & LBM_F_U) codes[n++] = 1;
  if (mask & LBM_F_T) codes[n++] = 2;
  if (mask & LBM_F_RHO) codes[n++] = 3;
  if (mask & LBM_F_VEL) { codes[n++] = 4; codes[n++] = 5; }
  if (mask & LBM_F_POP_PHI) for (int q = 0; q < D.qs; ++q) codes[n++] = 10 + q;
  if (mask & LBM_F_JU) { codes[n++] = 20; codes[n++] = 21; }
  if (mask & LBM_F_JT) { codes[n++] = 30; codes[n++] = 31; }
  if (mask & LBM_F_POP_F) for (int q = 0; q < 9; ++q) codes[n++] = 40 + q;
  if (mask & LBM_F_PEND_U) codes[n++] = 50;
  if (mask & LBM_F_PEND_T) codes[n++] = 51;
  if (mask & LBM_F_SPHI) for (int q = 0; q < D.qs - 1; ++q) codes[n++] = 60 + q;
  if (mask & LBM_F_SF) for (int q = 0; q < 8; ++q) codes[n++] = 70 + q;
  if (mask & LBM_F_SU) codes[n++] = 8;
  if (mask & LBM_F_ST) codes[n++] = 9;
  return n;
}

static std::string check_mask(const lbm_params& q, uint32_t mask) {
  if (mask == 0 || mask >= (1u << 15)) return "empty or unknown field mask";
  if ((mask & (LBM_F_U | LBM_F_JU | LBM_F_PEND_U | LBM_F_SU)) && !q.has_U) return "domain carries no U field";
  if ((mask & (LBM_F_T | LBM_F_JT | LBM_F_PEND_T | LBM_F_ST)) && !q.has_T) return "domain carries no T field";
  if ((mask & (LBM_F_RHO | LBM_F_VEL | LBM_F_POP_F | LBM_F_SF)) && !q.has_flow) return "domain carries no flow field";
  return "";
}

lbm_status lbm_read_fields(lbm_ctx* c, int32_t dom, uint32_t mask, int32_t dst_is_device, int32_t dst_fp64,
                           void* dst) {
  if (!c) return LBM_EINVAL;
  if (dom < 0 || dom >= c->ndom) return fail(c, LBM_EINVAL, "bad domain index");
  if (!dst) return fail(c, LBM_EINVAL, "dst is NULL");
  const std::string m = check_mask(c->P[dom], mask);
  if (!m.empty()) return fail(c, LBM_EINVAL, m);
  HIPCHK(c, hipSetDevice(c->device));
  const Dom& D = c->H[dom];
  int codes[kMaxCodes];
  const int nc = codes_for(D, mask, codes);
  const long long nsite = (long long)D.nx * D.ny * D.nz;
  HIPCHK(c, hipMemcpyAsync(c->d_codes, codes, sizeof(int) * nc, hipMemcpyHostToDevice, c->stream));
  const size_t esz = dst_fp64 ? 8 : 4;
  auto rd = [&](const int* cd, int cn, void* out) {
    if (c->dim == 3)
      c->ops3.read(D, c->stream, c->d_dom, c->k, cd, cn, dst_fp64, out);
    else
      c->ops.read(c->stream, c->d_dom, dom, c->k, cd, cn, dst_fp64, out, nsite);
  };
  if (dst_is_device) {
    rd(c->d_codes, nc, dst);
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
  }
  // host destination: stage in chunks of at most kStagePlanes planes
  for (int c0 = 0; c0 < nc; c0 += kStagePlanes) {
    const int cn = std::min(kStagePlanes, nc - c0);
    rd(c->d_codes + c0, cn, c->d_stage);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync((char*)dst + (size_t)c0 * nsite * esz, c->d_stage, (size_t)cn * nsite * esz,
                             hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_write_fields(lbm_ctx* c, int32_t dom, uint32_t mask, int32_t src_is_device, const void* src) {
  if (!c) return LBM_EINVAL;
  if (dom < 0 || dom >= c->ndom) return fail(c, LBM_EINVAL, "bad domain index");
  if (!src) return fail(c, LBM_EINVAL, "src is NULL");
  const std::string m = check_mask(c->P[dom], mask);
  if (!m.empty()) return fail(c, LBM_EINVAL, m);
  if ((mask & LBM_F_POP_PHI) && (mask & LBM_F_PHI))
    return fail(c, LBM_EINVAL, "phi is the sum of the phase populations: pass one of the two");
  if ((mask & LBM_F_POP_F) && (mask & (LBM_F_RHO | LBM_F_SF)))
    return fail(c, LBM_EINVAL, "rho is the sum of the flow populations: pass one of the two");
  if ((mask & LBM_F_POP_PHI) && (mask & LBM_F_SPHI))
    return fail(c, LBM_EINVAL, "pass either the phase populations or the stored phase planes");
  if (((mask & LBM_F_U) && (mask & LBM_F_SU)) || ((mask & LBM_F_T) && (mask & LBM_F_ST)))
    return fail(c, LBM_EINVAL, "pass either U (T) or its stored shift, not both");
  HIPCHK(c, hipSetDevice(c->device));
  const Dom& D = c->H[dom];
  int codes[kMaxCodes];
  const int nc = codes_for(D, mask, codes);
  const long long nsite = (long long)D.nx * D.ny * D.nz;
  HIPCHK(c, hipMemcpyAsync(c->d_codes, codes, sizeof(int) * nc, hipMemcpyHostToDevice, c->stream));
  auto wr = [&](const int* cd, int cn, const double* from) {
    if (c->dim == 3)
      c->ops3.write(D, c->stream, c->d_dom, c->k, cd, cn, from);
    else
      c->ops.write(c->stream, c->d_dom, dom, c->k, cd, cn, from, nsite);
  };
  if (src_is_device) {
    wr(c->d_codes, nc, (const double*)src);
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
  }
  // host source: stage chunks of at most kStagePlanes planes, never splitting the
  // population groups (their planes are re-encoded together)
  const int stage_planes = (int)(c->stage_elems / (size_t)nsite);
  int c0 = 0;
  while (c0 < nc) {
    int c1 = c0;
    while (c1 < nc) {
      const int unit = (codes[c1] == 10) ? D.qs : (codes[c1] == 40) ? (c->dim == 3 ? 19 : 9) : 1;
      if (c1 + unit - c0 > std::min(kStagePlanes, stage_planes)) break;
      c1 += unit;
    }
    if (c1 == c0) return fail(c, LBM_EINVAL, "staging buffer too small for one field group");
    HIPCHK(c, hipMemcpyAsync(c->d_stage, (const double*)src + (size_t)c0 * nsite,
                             sizeof(double) * (size_t)(c1 - c0) * nsite, hipMemcpyHostToDevice, c->stream));
    wr(c->d_codes + c0, c1 - c0, c->d_stage);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c0 = c1;
  }
  return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->h_diag) (void)hipHostFree(c->h_diag);
  if (c->h_first) (void)hipHostFree(c->h_first);
  if (c->h_front) (void)hipHostFree(c->h_front);
  delete c;
}

}  // extern "C"
