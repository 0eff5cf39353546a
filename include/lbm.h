/*
 * lbm.h -- C ABI of the multirate MRT lattice-Boltzmann hot path for
 * thermosolutal dendritic solidification (phase field with anisotropic
 * streaming and anti-trapping current, concentration, temperature, flow),
 * built for AMD MI355X (gfx950).
 *
 * The method (paper: "A unified multirate lattice Boltzmann framework for
 * thermosolutal dendritic solidification"):
 *   - every field chi in {phi, U, T, F} is carried by its own distributions
 *     and collides with the moment-space MRT operator of Eq. (14);
 *   - field chi advances with its own step dt_chi = N_chi * dt_base
 *     (Eq. 34) and relaxation times scale with dt_chi (Eq. 24, 32);
 *   - after every phase update the resolved increment dphi (Eq. 36) is
 *     turned into solute and latent-heat increments (Eq. 37-38) that are
 *     injected at once into U and T (Eq. 39).
 *
 * Conventions for every entry point:
 *   - Lattice units: dx = 1; time in the unit of dt_base.
 *   - Grids are x-fastest; 2D domains have nz = 1.
 *   - Every call returns an lbm_status; no exception crosses the ABI;
 *     lbm_last_error() returns the text of the last failure of a context.
 *   - All device work is issued on the stream passed to lbm_create (NULL =
 *     the default stream).  lbm_step_multirate (which reads the device's
 *     non-finite screen at its end), lbm_read_fields to host memory and
 *     lbm_write_fields from host memory synchronise with that stream.
 *   - The library allocates device memory only inside lbm_create (and only
 *     when no workspace is supplied) and frees it only in lbm_destroy.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument: tau <= 1/2, N_chi < 1, bad sizes, ... */
  LBM_ENOMEM = -2,     /* device allocation failed or workspace too small     */
  LBM_EDEVICE = -3,    /* a HIP call failed                                   */
  LBM_EUNSTABLE = -4,  /* non-finite values were found in the state           */
  LBM_ESTATE = -5      /* call not valid in the current state                 */
} lbm_status;

/* Field selection masks for lbm_read_fields / lbm_write_fields.  Planes are
 * packed in the order of the bits below (lowest bit first), each plane
 * nx*ny*nz values, x fastest. */
enum {
  LBM_F_PHI = 1 << 0,    /* phi                                   (1 plane)  */
  LBM_F_U = 1 << 1,      /* U                                     (1 plane)  */
  LBM_F_T = 1 << 2,      /* T                                     (1 plane)  */
  LBM_F_RHO = 1 << 3,    /* flow density                          (1 plane)  */
  LBM_F_VEL = 1 << 4,    /* flow velocity u_x, u_y[, u_z]         (dim)      */
  LBM_F_POP_PHI = 1 << 5,/* phase populations f_0..f_{Q-1}        (Q)        */
  LBM_F_JU = 1 << 6,     /* first moment of the U populations     (dim)      */
  LBM_F_JT = 1 << 7,     /* first moment of the T populations     (dim)      */
  LBM_F_POP_F = 1 << 8,  /* flow populations f_0..f_{QF-1}        (QF)       */
  LBM_F_PEND_U = 1 << 9, /* pending U increments (accumulated coupling)      */
  LBM_F_PEND_T = 1 << 10,/* pending T increments (accumulated coupling)      */
  LBM_F_SPHI = 1 << 11,  /* stored phase planes s_i = f_i - w_i phi, i>=1 (4) */
  LBM_F_SF = 1 << 12,    /* stored flow planes s_i = f_i - w_i rho, i>=1  (8) */
  LBM_F_SU = 1 << 13,    /* stored U plane U - U0                 (1 plane)  */
  LBM_F_ST = 1 << 14     /* stored T plane T - T0                 (1 plane)  */
};
/* (In 3D the population groups hold 7 and 19 planes and SPHI / SF 6 and 18.)
 * The U and T planes are kept as the shifts U - U0 and T - T0 from the
 * initial values, so that FP32 keeps the small far-field increments; U and
 * T read and write absolute values, SU and ST the stored shifts.
 * A checkpoint that restores bit for bit is the set
 * PHI | SU | ST | RHO | VEL | JU | JT | PEND_U | PEND_T | SPHI | SF
 * (the fields a domain carries), read and written back as FP64. */

/* boundary kinds, per axis */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1, LBM_BC_INLET_OUTFLOW = 2 };
/* population storage formats (collision arithmetic is FP64 for F64, else FP32) */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16 = 2, LBM_STORE_BF16 = 3 };
/* phase-change coupling: Eq. (39) at every phase step, or the delayed
 * variant that sums increments and injects them after the field's next
 * transport update (the ablation of Section 4.4) */
enum { LBM_COUPLE_INSTANT = 0, LBM_COUPLE_ACCUM = 1 };
/* temperature field: transported with latent heat (Eq. 10-12, 38); the
 * pulled profile of 3D directional solidification (advected at V_pull along
 * z, no latent heat, z walls held at the moving linear profile); or the cold
 * bottom of Section 4.4 (transported with latent heat, the low wall of the
 * last axis held at T0; that axis must have walls) */
enum { LBM_T_TRANSPORT = 0, LBM_T_PULLED = 1, LBM_T_DIRICHLET_LOW = 2 };
/* grad phi for the normal, a_s and N of the phase collision: the isotropic
 * finite-difference stencil (ISO), or Eq. (40) on the phase populations with
 * the equilibrium flux v_n dt and tau_phi of the site's previous phase step
 * (EQ40, 2D; the first step sees the initial equilibrium, v_n = 0 and
 * A = 1).  The transfer's normal (Eq. 37) and the transport sources keep the
 * stencil in both.  EQ40 runs on the tiled phase kernel (no marching,
 * deferred or fused transfer), and its lagged planes are not part of the
 * checkpoint masks. */
enum { LBM_GRAD_ISO = 0, LBM_GRAD_EQ40 = 1 };

/* Parameters of one domain (host memory, FP64, lattice units).  Field
 * names follow the paper's notation. */
typedef struct {
  int32_t dim;            /* 2, or 3 (single-domain contexts only)           */
  int32_t nx, ny, nz;     /* grid size; nz = 1 in 2D                         */
  int32_t q_scalar;       /* scalar lattice: 5 (D2Q5) in 2D, 7 (D3Q7) in 3D  */
  int32_t has_U, has_T, has_flow;
  int32_t N_phi, N_U, N_T, N_F;         /* update factors (Eq. 34), >= 1     */
  double dt_base;                       /* baseline step (Eq. 34)            */
  double W0, tau0, eps_s, lam, Mc, k, theta_c;   /* Eq. (1)-(5); theta_c:
                                           crystal orientation [rad]        */
  double D_L, D_S, C_inf;               /* Eq. (5), (7)                      */
  double kappa_S, kappa_L, rhoCp_S, rhoCp_L;     /* Eq. (11)                 */
  double rho_L, L_h, T_m, m_L, Cp_L;    /* Eq. (5), (12)                     */
  double nu, s_e, s_eps, s_q, u_in;     /* Eq. (27)-(32)                     */
  double Fb[3];                         /* body force (Eq. 13, 27, 30)       */
  int32_t bc[3];                        /* scalar boundaries per axis        */
  int32_t flow_bc[3];                   /* flow boundaries per axis          */
  double U0, T0;                        /* initial uniform U and T           */
  int32_t u0_liquid_only;               /* initial u = u_in (1 - phi)/2 x^  */
  int32_t coupling;                     /* LBM_COUPLE_*                      */
  int32_t T_mode;                       /* LBM_T_TRANSPORT, _PULLED, _DIRICHLET_LOW */
  int32_t grad_phi;                     /* LBM_GRAD_ISO or LBM_GRAD_EQ40       */
  double T_grad, V_pull, z_front;       /* pulled temperature (3D):
                                           T0 + T_grad (z - z_front - V_pull t);
                                           z_front: mean height of the front
                                           set by lbm_init_front */
} lbm_params;

/* Per-domain diagnostics (FP64 reductions on the device; Section 4.4
 * defines S_phi, J_U, M_C and R_M).  In 3D, tip[0] is the highest and
 * tip[1] the mean phi = 0 crossing height over columns. */
typedef struct {
  int64_t step;            /* base steps completed                           */
  double solid;            /* sum (1 + phi)/2                                */
  double M_C;              /* sum C, C = C_inf kfac(phi)[1+(1-k)U]/2 (Eq. 5) */
  double enthalpy;         /* sum (T - rho_L L_h phi / (2 rhoCp_L))          */
  double mass;             /* sum rho                                        */
  double S_phi;            /* max |dU_pc| of the last phase step             */
  double J_U;              /* max |U_post - U_pre| of the last injection     */
  double tip[16];          /* tip distances: 4 axes for each of <= 4 seeds   */
  int64_t nonfinite;       /* count of non-finite phi/U/T/rho values         */
  double t;                /* time: step * dt_base                           */
  double R_M;              /* [M_C(t) - M_C(0)] / M_C(0), M_C(0) taken at the
                              first lbm_step_multirate after initialisation
                              (0 for a domain without U)                     */
  int64_t first_nonfinite_step; /* first base step at whose screen a
                              non-finite phi/U/T/rho value was found, or -1  */
} lbm_diag;

/* Device bytes a context needs for these domains (states with their buffers,
 * descriptors, tile lists, reduction partials).  Not an operation of the
 * method: it sizes the caller-owned workspace of lbm_create, which holds
 * the fields the paper's Section 3 defines (distributions of Eq. 14-33 per
 * carried field, plus the pending increments of the Section 4.4 ablation).
 * 0 on invalid input. */
size_t lbm_workspace_bytes(const lbm_params* p, int32_t n_domains, int32_t storage);

/* Create a context for n_domains domains that are stepped together.
 *   p            host array of n_domains parameter sets (copied)
 *   storage      LBM_STORE_* population storage (one for all domains)
 *   device       HIP device ordinal
 *   hip_stream   hipStream_t to issue work on (NULL = default stream)
 *   workspace    device buffer of >= lbm_workspace_bytes() bytes, owned by
 *                the caller and kept alive until lbm_destroy; NULL makes the
 *                library allocate (and later free) it
 * Errors: LBM_EINVAL (a relaxation time <= 1/2 at phi = +-1, N_chi < 1,
 * unsupported lattice, sizes), LBM_ENOMEM, LBM_EDEVICE.  On error *out is
 * NULL.  The state is left uninitialised until lbm_init_seeds. */
lbm_status lbm_create(const lbm_params* p, int32_t n_domains, int32_t storage,
                      int32_t device, void* hip_stream, void* workspace,
                      size_t workspace_bytes, lbm_ctx** out);

/* Initialise one domain: phi = max over seeds of tanh[(R_s - r)/(sqrt2 W0)]
 * (Section 4.1), U = U0, T = T0, rho = 1, u = 0 or u_in (1 - phi)/2 along x,
 * every population at equilibrium with v_n = 0.  Resets the step counter.
 *   centres  host, n_seeds * dim doubles (x, y[, z]) in lattice units
 *   radii    host, n_seeds doubles
 * Seeds (<= 4 per domain) are also the origins of the tip diagnostics. */
lbm_status lbm_init_seeds(lbm_ctx* ctx, int32_t domain, int32_t n_seeds,
                          const double* centres, const double* radii);

/* Initialise a domain with a planar solid layer along its last axis:
 * phi = tanh[(z_front + xi - z)/(sqrt2 W0)] with z = y in 2D (Eq. 41 with
 * xi = sin(10 pi x / L)) and z in 3D (a random form of Eq. 41), U = U0,
 * T = T0 or the pulled profile, flow at rest (3D) or u0 as for seeds (2D),
 * populations at equilibrium.
 *   xi  host, column offsets: nx values in 2D, nx * ny (x fastest) in 3D,
 *       or NULL for a flat front.
 * Resets the step counter. */
lbm_status lbm_init_front(lbm_ctx* ctx, int32_t domain, const double* xi);

/* Advance every domain by n_base_steps base steps of Eq. (34): at base
 * step k a field runs iff k mod N_chi == 0, in the order phase (+ the
 * transfer of Eq. 36-39), U, T, flow.  Whole multirate cycles are replayed
 * from a captured HIP graph.
 * Failure detection: the phi, U, T and rho planes of every domain are
 * screened for non-finite values on the device after every replayed cycle
 * and after the call's last step; the call synchronises at its end and
 * returns LBM_EUNSTABLE (with the domain and step in lbm_last_error) once
 * any screen has failed since the domain's initialisation.  The state is
 * left readable.
 * If diag_out is non-NULL, diagnostics of every domain are reduced after the
 * last step and written to diag_out[0..n-1]; LBM_EUNSTABLE is then also
 * returned when the reduction counts non-finite values.  The first call
 * after an initialisation also reduces M_C(0) for R_M. */
lbm_status lbm_step_multirate(lbm_ctx* ctx, int64_t n_base_steps, lbm_diag* diag_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * stepping as lbm_step_multirate, with the same kernels and the same
 * results, that allocates nothing.  The reduction scratch of its kernels
 * (per-tile partials, per-run maxima, the reduced diagnostics, the 3D front
 * partials) lives in a static device array of 16 MiB per GPU, held until
 * the process ends, instead of the context's workspace; no HIP graph is
 * captured or replayed (every step is launched directly) and the tile-height
 * autotuner does not run (a height fixed by lbm_configure is used, else
 * 16 rows until an lbm_step_multirate call has tuned it).
 * Limits and semantics:
 *   - LBM_EINVAL when the context's scratch exceeds the static array (a
 *     2D context with more than about 200,000 64 x 4 tiles, a 3D domain of
 *     more than about 50 M sites);
 *   - the array is shared by every call on a GPU and keeps the last call's
 *     contents: each call clears its partials first, so S_phi and J_U report
 *     the phase steps and injections of this call only (n_base_steps >= 1,
 *     and with accumulated coupling at least one U update, for a defined
 *     J_U); calls that overlap on one GPU (several streams or threads) race;
 *   - failure detection and its synchronisation at the end of the call are
 *     those of lbm_step_multirate. */
lbm_status lbm_step_multirate_static(lbm_ctx* ctx, int64_t n_base_steps, lbm_diag* diag_out);

/* Copy the planes selected by mask of one domain into dst (caller-owned,
 * device memory if dst_is_device else host memory), as FP64 if dst_fp64
 * else FP32, packed in mask-bit order.  Populations are reconstructed from
 * the stored representation, whose zeroth moments are the macroscopic
 * fields of Eq. (18) and (27): f_0 = w_0 chi - sum_{i>0} s_i with chi = phi
 * (U, T) and the stored deviations s_i = f_i - w_i chi, and likewise for
 * the flow with rho; the first moments of U and T are stored as such.
 * Errors: LBM_EINVAL (bad domain, NULL dst, a mask naming a field the
 * domain does not carry), LBM_EDEVICE.  Synchronises when dst is host
 * memory. */
lbm_status lbm_read_fields(lbm_ctx* ctx, int32_t domain, uint32_t mask,
                           int32_t dst_is_device, int32_t dst_fp64, void* dst);

/* Overwrite the planes selected by mask of one domain from src (same
 * packing as lbm_read_fields, FP64).  Used for checkpoint restore and to
 * inject faults in tests.  Populations are given in full and re-encoded
 * into the stored representation, their sums becoming the macroscopic
 * fields of Eq. (18) and (27): LBM_F_POP_PHI requires LBM_F_PHI to be
 * absent (phi is the sum of the populations), LBM_F_POP_F requires RHO and
 * SF to be absent.  Errors: LBM_EINVAL (as for lbm_read_fields, or a
 * conflicting mask), LBM_EDEVICE.  Synchronises when src is host memory. */
lbm_status lbm_write_fields(lbm_ctx* ctx, int32_t domain, uint32_t mask,
                            int32_t src_is_device, const void* src);

/* Tuning: rows per tile of the stencil kernels (4, 8, 16 or 32; 0 = autotune;
 * in 3D, rows of every kernel's 64-wide tiles, 4 or 8 (the flow keeps 4 in
 * FP64), or 0: the autotuner times the phase kernel, the flow and (with
 * N_phi = 1 and instantaneous coupling) the transfer, and with N_U = 1 as
 * well the U transport, at both heights and six z-run lengths at the next
 * lbm_step_multirate and keeps the fastest of each (with the environment
 * variable LBM_AUTOTUNE_LOG set, the times and picks go to stderr); the
 * other transports take measured defaults (8 rows); every choice gives the
 * same bits) and flags:
 *   LBM_CFG_GRAPH           replay whole multirate cycles from a HIP graph
 *   LBM_CFG_FUSE_TRANSFER   2D: run the transfer of Eq. (36)-(39) inside the
 *                           phase kernel, which then recomputes a halo of
 *                           three sites (domains of at least 8 x 8; results
 *                           bitwise identical to the separate kernels; slower
 *                           on MI355X at every size measured, so off by default)
 *   LBM_CFG_MARCH           2D: the phase, transfer and T-transport kernels
 *                           always walk 64-wide columns up in runs of 64
 *                           rows instead of tiling them (domains of at least
 *                           16 x 16; results bitwise identical to the tiles;
 *                           the U transport stays tiled)
 *   LBM_CFG_TILES           2D: every kernel tiles
 * With neither of the last two, the kernels march when every domain is at
 * least 16 x 16 and the context holds at least 1024 column runs (enough
 * blocks to fill the chip), and tile otherwise.
 *   LBM_CFG_NO_DEFER        2D: never defer a transfer.  Otherwise, in a
 *                           tiled D2Q5 context with N_phi = 1, instantaneous
 *                           coupling and domains of at least 8 x 8, the
 *                           transfer of a phase step at which no transport
 *                           runs (and which is not the last step of a call
 *                           or of a graph cycle) runs inside the next phase
 *                           kernel, and where every domain has U in one
 *                           update group, the transfer of a step at which U
 *                           is due runs inside that U transport.  In a
 *                           marching context whose domains all have a
 *                           transported T (instantaneous coupling, one
 *                           update group), the transfer of a step at which
 *                           T is due runs inside that T transport.  Results
 *                           bitwise identical.
 *   LBM_CFG_QUEUE           2D marching kernels: launch as many blocks as fit
 *                           on the chip and let them take the column runs from
 *                           eight per-XCD work queues (whole domains per
 *                           queue, largest first; an idle block takes runs
 *                           from the other queues); results bitwise
 *                           identical to the static grids
 *   LBM_CFG_GRID            2D marching kernels: one block per run, static grid
 * With neither, the autotuner times the marching phase kernel in both forms
 * and keeps the faster.
 * Default after lbm_create: autotune, LBM_CFG_GRAPH.  Unknown flags,
 * LBM_CFG_MARCH with LBM_CFG_TILES, or LBM_CFG_QUEUE with LBM_CFG_GRID:
 * LBM_EINVAL. */
enum { LBM_CFG_GRAPH = 1, LBM_CFG_FUSE_TRANSFER = 2, LBM_CFG_MARCH = 4, LBM_CFG_TILES = 8, LBM_CFG_NO_DEFER = 16,
       LBM_CFG_QUEUE = 32, LBM_CFG_GRID = 64 };
lbm_status lbm_configure(lbm_ctx* ctx, int32_t tile_rows, int32_t flags);

/* Average device time, in milliseconds, of one launch of each kernel kind
 * over every domain, measured with HIP events around `reps` back-to-back
 * launches on the context stream: ms_out[0] phase, [1] transfer, [2] U
 * transport, [3] T transport, [4] flow, [5] the phase kernel carrying the
 * previous step's deferred transfer, [6] the U transport carrying its
 * step's transfer, [7] the marching T transport carrying its step's
 * transfer (-1 where the context has no such kernel); the arrays hold 8
 * values.  per_step_out[0..7] (may be NULL) receives the fraction of that
 * time spent per base step (each group of domains sharing an update factor
 * N contributes 1/N of its own launch time; with deferred transfers the
 * plain phase, transfer, U and T kernels run on the other steps), so
 * ms_out * per_step_out is the device time per base step.  The timing launches overwrite the state:
 * every domain must be re-initialised with lbm_init_seeds before the next
 * lbm_step_multirate. */
lbm_status lbm_kernel_times(lbm_ctx* ctx, int32_t reps, double* ms_out, double* per_step_out);

/* Base steps completed since the last lbm_init_seeds. */
int64_t lbm_steps_done(const lbm_ctx* ctx);

/* 1 when the context's 2D phase, transfer and T-transport kernels march up
 * column runs (see lbm_configure), 0 when they tile or the context is 3D,
 * -1 for ctx NULL. */
int32_t lbm_marching(const lbm_ctx* ctx);

/* Tile height of the 2D tiled kernels in use: the one fixed by
 * lbm_configure, else the autotuner's pick once it has run (at the first
 * lbm_step_multirate or lbm_kernel_times), else 0; for a 3D context the
 * rows fixed by lbm_configure, 0 for the per-kernel defaults; -1 for ctx
 * NULL. */
int32_t lbm_tile_rows(const lbm_ctx* ctx);

/* Text of the last error of ctx (or of the last failed lbm_create when ctx
 * is NULL).  Owned by the library. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Release the context and, if the library allocated it, the workspace. */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
