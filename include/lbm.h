/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q37 thermal lattice Boltzmann
 * library, liblbm.so.
 *
 * The method is the one of Calore, Gabbana, Schifano, Tripiccione,
 * "Optimization of Lattice Boltzmann Simulations on Heterogeneous Computers"
 * (arXiv:1703.04594), section 3: populations f_l on a 2-D lattice evolve by
 * the BGK equation, eq. (1); density, velocity and temperature are the
 * moments of eq. (2); one time step is the pull streaming of eq. (4)
 * ("propagate"), the wall boundary condition ("bc") on the three lowest and
 * three highest rows, and the collision ("collide"), run in that order
 * (section 5, control flow of one time step).
 *
 * Model readings where the paper defers to its model references:
 *  - 37 hops e_l with |e|^2 in {0,1,2,4,5,8,9,10} (every hop at most 3 sites),
 *    canonical order by |e|^2 then angle in [0, 2 pi) -- lbm_velocity_table;
 *  - xi_l = c e_l, weights and c from the 8th-order Gaussian moment equations;
 *  - f^eq: 4th-order Hermite expansion of the Maxwellian in D = 2;
 *  - gravity g = (0, g_y) by shifting the equilibrium: u* = u + tau g,
 *    T* = T + tau (1 - tau) g_y^2 / 2;
 *  - walls: after propagate, each slot of the 3 bottom (top) rows whose pull
 *    source lies below (above) the lattice receives f^eq_l(1, 0, T_wall) times
 *    the pre-propagate density of the fluid site mirroring that source across
 *    the wall (row -1-k <-> row k; row LY+k <-> row LY-1-k); x is periodic.
 *
 * Conventions
 *  - Every array pointer is a DEVICE pointer owned by the caller (for
 *    instance the data_ptr() of a torch tensor on the same device), unless a
 *    parameter says "host".  Lattice contexts never allocate device memory:
 *    all of their buffers live in the caller's workspace (the co-execution
 *    calls and lbm_conservation_noalloc state their own exceptions).
 *  - Field arrays are [lx][ly], y fastest, FP64.
 *  - "Canonical" population arrays are [37][lx][ly], y fastest, in the storage
 *    precision: FP64 populations f_l for LBM_FP64; FP32 deviations
 *    f_l - w_l for both FP32 forms.
 *  - "State" arrays hold one population buffer in the library's internal
 *    padded layout (lbm_state_bytes bytes); they are opaque, for snapshots.
 *  - All calls enqueue work on the stream given to lbm_create and return
 *    without waiting.  Argument and state errors are reported at once; a
 *    failed launch returns LBM_ERR_HIP; faults of running kernels surface at
 *    lbm_sync or at a later call.  lbm_last_error gives the message.
 *  - A context belongs to the device that is current at lbm_create (that of
 *    its workspace and stream; its launch settings are chosen for that
 *    device).  Every later call on the context is made with that device
 *    current.
 *  - A context is used by one host thread at a time.  Two contexts may share
 *    nothing but the device.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_NPOP 37

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = 1,  /* bad argument or parameter                      */
    LBM_ERR_SIZE = 2,     /* workspace too small                            */
    LBM_ERR_HIP = 3,      /* a HIP call or kernel launch failed             */
    LBM_ERR_STATE = 4     /* call not allowed in the context's current state */
} lbm_status;

/* Population storage and collide arithmetic.  LBM_FP64: FP64 populations,
 * FP64 arithmetic.  LBM_FP32_SHIFTED: FP32 deviations f_l - w_l from the
 * rest state, collided in FP32 with the moment sums (37 terms each, before
 * and after the relaxation) accumulated in FP64.  LBM_FP32_SHIFTED_F32SUMS:
 * the same storage and collision with those sums in FP32 as well.  Both FP32
 * forms keep FP64 for lbm_conservation and lbm_get_macros. */
typedef enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1, LBM_FP32_SHIFTED_F32SUMS = 2 } lbm_precision;
typedef enum { LBM_Y_WALLS = 0, LBM_Y_PERIODIC = 1 } lbm_ybc;
/* How x-periodicity reaches propagate: wrap the source column index inside the
 * kernel, or first copy 3-column halos (the in-GPU form of the paper's halo
 * exchange between lattice regions, section 5). Results are identical. */
typedef enum { LBM_X_WRAP = 0, LBM_X_HALO = 1 } lbm_xmode;
/* lbm_step as three kernels (propagate, bc, collide) or as one fused
 * gather-collide pass (eq. (4) evaluated per site). Results are identical up
 * to rounding order (none: both evaluate the same expressions). */
typedef enum { LBM_STEP_SPLIT = 0, LBM_STEP_FUSED = 1 } lbm_step_kind;
/* Population storage.  Both keep every (population, column) segment
 * contiguous in y with 128-byte aligned rows (the paper's column-major
 * order, section 4): PLANES stores population l of all columns together
 * (structure of arrays); COLUMNS stores the 37 segments of a column together,
 * so the 37 streams a site touches lie within one column (better DRAM
 * locality).  Results are identical. */
typedef enum { LBM_LAYOUT_PLANES = 0, LBM_LAYOUT_COLUMNS = 1 } lbm_layout;

typedef struct {
    int32_t lx, ly;        /* lattice sites; lx >= 7, ly >= 7               */
    int32_t precision;     /* lbm_precision                                  */
    int32_t ybc;           /* lbm_ybc                                        */
    int32_t xmode;         /* lbm_xmode                                      */
    int32_t step_kind;     /* lbm_step_kind                                  */
    int32_t adjoint;       /* 0: none; 1: adjoint buffers with FP64 lambda;  */
                           /* 2: FP32 lambda storage (arithmetic, d/dtau and */
                           /*    dL/dP stay FP64)                            */
    int32_t layout;        /* lbm_layout                                     */
    double tau;            /* relaxation time, > 0.5                         */
    double g_y;            /* gravity, lattice units per step (y component)  */
    double t_bottom;       /* wall temperatures (ignored for LBM_Y_PERIODIC) */
    double t_top;
} lbm_params;

/* Rayleigh-Taylor initial profile: T0(x,y) = t_mid - t_amp *
 * tanh((y - y_mid - P(x,y)) / width), rho0 = p0 / T0, u0 = 0. */
typedef struct {
    double t_mid, t_amp, p0, width, y_mid;
} lbm_rt_profile;

/* ---- sizes and lifetime -------------------------------------------------- */

/* Bytes of device workspace lbm_create needs; 0 if *p is invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);
/* Bytes of one opaque state snapshot; 0 if *p is invalid. */
size_t lbm_state_bytes(const lbm_params* p);

/* Validates *p (lx, ly >= 7, lx * ly <= 2^31, tau > 0.5 and finite, finite
 * g_y, known enums, adjoint 0, 1 or 2; else LBM_ERR_INVALID, and
 * LBM_ERR_SIZE if bytes is too small) and binds
 * a context to dev_workspace (>= lbm_workspace_bytes(p) bytes, 256-byte
 * aligned, caller-owned, must outlive the context) and hip_stream (a
 * hipStream_t, or NULL for the default stream).  Zeroes the workspace.  The
 * context holds host-side metadata only. */
lbm_status lbm_create(const lbm_params* p, void* dev_workspace, size_t bytes,
                      void* hip_stream, lbm_ctx** out);
/* Frees the host-side context; never touches the workspace. NULL is a no-op. */
void lbm_destroy(lbm_ctx* ctx);
/* Changes tau (> 0.5) for subsequent collide and adjoint calls. */
lbm_status lbm_set_tau(lbm_ctx* ctx, double tau);

/* ---- initial state ------------------------------------------------------- */

/* f = f^eq(rho, (ux, uy), T) at every site (eq. (2)'s moments of the
 * result are the given fields).  Fields: device FP64 [lx][ly]. */
lbm_status lbm_init(lbm_ctx* ctx, const double* rho, const double* ux,
                    const double* uy, const double* T);
/* f = f^eq of the Rayleigh-Taylor profile *prof (host struct) displaced by
 * the device FP64 field P [lx][ly]. */
lbm_status lbm_init_rt(lbm_ctx* ctx, const double* P, const lbm_rt_profile* prof);

/* ---- the time step (section 5 order: propagate, bc, collide) -------------- */

/* Pull streaming, eq. (4): next_l(x, y) = cur_l(x - ex_l, y - ey_l) for every
 * population and site, x periodic (y periodic for LBM_Y_PERIODIC).  Writes
 * the other buffer, which becomes current; the old one is kept for lbm_bc. */
lbm_status lbm_propagate(lbm_ctx* ctx);
/* Wall rule (see above) on the current buffer, reading the buffer before the
 * last propagate.  No-op for LBM_Y_PERIODIC.  LBM_ERR_STATE if no propagate
 * has run since the state was set. */
lbm_status lbm_bc(lbm_ctx* ctx);
/* BGK collision, eq. (1) with dt = 1, in place on the current buffer:
 * moments (eq. (2)), gravity shift, equilibrium, f <- f + (f^eq - f)/tau. */
lbm_status lbm_collide(lbm_ctx* ctx);
/* n >= 0 times (propagate, bc, collide), split or fused per step_kind.
 * It only launches kernels on the context's stream, so it can be captured
 * into a HIP graph there (after at least one eager step).  A replay repeats
 * the captured launches with the buffers they were captured with: capture an
 * even n, which ends on the buffers it started from, and each replay then
 * advances the state by n steps, bitwise as n eager steps would. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* ---- read-out and snapshots ---------------------------------------------- */

/* Moments of eq. (2) of the current state, computed in FP64: rho,
 * u = sum xi f / rho, T = sum |xi - u|^2 f / (2 rho).  Device FP64 [lx][ly]. */
lbm_status lbm_get_macros(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* T);
/* Canonical population copies (device, storage precision). set_pops clears
 * the "previous buffer" so lbm_bc needs a propagate first. */
lbm_status lbm_get_pops(lbm_ctx* ctx, void* dst);
lbm_status lbm_set_pops(lbm_ctx* ctx, const void* src);
/* Opaque snapshots, lbm_state_bytes each (device): the padded population
 * buffer followed by the densities of its 3 rows next to each wall. */
lbm_status lbm_get_state(lbm_ctx* ctx, void* dst);
lbm_status lbm_set_state(lbm_ctx* ctx, const void* src);
/* One time step (section 5: propagate, bc, collide; evaluated as the pull of
 * eq. (4) per site, identical to lbm_step) from one snapshot into another:
 * dst_state <- step(src_state).  Both are device buffers of lbm_state_bytes,
 * 256-byte aligned, not overlapping, in the format of lbm_get_state (dst
 * receives the new state's wall densities too, so it can serve as the next
 * source or as an lbm_adjoint_step snapshot).  The sites and wall densities
 * of src_state are only read; its padding (y ghost rows, x halo columns) is
 * refreshed in place when the boundary mode needs it.  The context's own
 * population buffers are not touched.  Lets a checkpointed replay run from
 * snapshot to snapshot instead of stepping the context and copying its state
 * out. */
lbm_status lbm_step_state(lbm_ctx* ctx, void* src_state, void* dst_state);
/* Lattice totals of the collision invariants, accumulated in FP64 with a
 * fixed reduction order (bitwise reproducible): out4 = {sum rho, sum j_x,
 * sum j_y, sum E}, E = sum_l |xi_l|^2 f_l.  dev_out4: device FP64 [4]. */
lbm_status lbm_conservation(lbm_ctx* ctx, double* dev_out4);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the totals
 * of lbm_conservation for a canonical population array, with no context and
 * no workspace.  The reduction's block partials live in a fixed device array
 * of the library (1024 x 4 doubles = 32 KiB; each GPU the library runs on
 * holds its own copy until the process ends); nothing is allocated per call
 * and nothing needs clearing, since every partial is rewritten by each call.
 * Calls that overlap on one GPU (different streams, or host threads) race on
 * that array; calls are ordered by the stream.
 *   precision:  lbm_precision of pops (FP64 f_l, or FP32 deviations f_l - w_l
 *               for either FP32 form)
 *   lx, ly:     >= 1 each, lx * ly <= LBM_NOALLOC_MAX_SITES (else LBM_ERR_SIZE)
 *   pops:       device canonical [37][lx][ly] array, only read
 *   dev_out4:   device FP64 [4] <- {sum rho, sum j_x, sum j_y, sum E}, with
 *               the same kernels and reduction order as lbm_conservation, so
 *               the two give bitwise equal totals for equal states
 *   hip_stream: a stream of the current device (NULL: its null stream)
 * Runs on the current device.  Errors: LBM_ERR_INVALID / LBM_ERR_SIZE before
 * anything is launched, LBM_ERR_HIP for a failed lookup or launch; the
 * message is lbm_last_error(NULL). */
#define LBM_NOALLOC_MAX_SITES (1LL << 31)
lbm_status lbm_conservation_noalloc(int precision, int lx, int ly, const void* pops, double* dev_out4,
                                    void* hip_stream);

/* ---- adjoint (requires params.adjoint != 0) ------------------------------- */
/* The adjoint state lambda = dL/df (one value per population and site; stored
 * in FP64, or FP32 when params.adjoint == 2) lives in the workspace.  A
 * reverse sweep is: seed lambda_N, then for n = N-1 .. 0 call
 * lbm_adjoint_step with the forward state f_n, then lbm_adjoint_init_rt for
 * dL/dP (and lbm_adjoint_take_dtau for dL/dtau if the steps deferred it). */

/* lambda <- dL/df of L = 1/2 sum (T - T_target)^2 at the current state;
 * *dev_loss (device FP64 scalar) <- L.  T_target: device FP64 [lx][ly]. */
lbm_status lbm_loss_temperature(lbm_ctx* ctx, const double* T_target, double* dev_loss);
/* lambda <- sum_{x,y} dT(x,y) dT(x,y)/df at the current state: the adjoint
 * seed for an arbitrary upstream gradient dT of the temperature field. */
lbm_status lbm_adjoint_seed_temperature(lbm_ctx* ctx, const double* dT);
/* One reverse step: with f_n (a device state snapshot, lbm_state_bytes,
 * 256-byte aligned, as written by lbm_get_state or lbm_step_state after n
 * forward steps of a context with the same parameters) and lambda_{n+1} in the
 * context, replaces lambda by lambda_n = (d step / d f_n)^T lambda_{n+1}
 * (collide^T, bc^T and propagate^T) and adds lambda_{n+1} . d step/d tau to
 * *dev_dtau_acc (device FP64 scalar).  The snapshot is only read; the
 * population buffers are not touched.  Internally the context keeps the
 * step's collide^T output and applies bc^T and propagate^T when lambda_n is
 * next read (by the next reverse step, lbm_adjoint_init_rt or
 * lbm_adjoint_get_lambda), so those reads see lambda_n exactly.
 * dev_dtau_acc may be NULL: the step's d/dtau term is then added to sums the
 * context keeps per block of sites (no reduction kernel for this step), and
 * lbm_adjoint_take_dtau later adds all such terms to a scalar at once. */
/* Errors: LBM_ERR_STATE without adjoint buffers or before lambda is seeded,
 * LBM_ERR_INVALID for a NULL or misaligned snapshot. */
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* f_n_state, double* dev_dtau_acc);
/* *dev_dtau_acc (device FP64 scalar) += the d/dtau terms of every
 * lbm_adjoint_step called with a NULL accumulator since the context was
 * created or last taken from, then those sums restart at zero.  Summed per
 * block over steps, then over blocks, in a fixed order: reproducible, and
 * equal to per-step accumulation up to rounding. */
lbm_status lbm_adjoint_take_dtau(lbm_ctx* ctx, double* dev_dtau_acc);
/* dP <- dL/dP for the initial state of lbm_init_rt(P, prof), from lambda_0. */
lbm_status lbm_adjoint_init_rt(lbm_ctx* ctx, const double* P,
                               const lbm_rt_profile* prof, double* dP);
/* Canonical FP64 [37][lx][ly] copies of lambda (device). */
lbm_status lbm_adjoint_get_lambda(lbm_ctx* ctx, double* dst);
lbm_status lbm_adjoint_set_lambda(lbm_ctx* ctx, const double* src);

/* ---- layout study ---------------------------------------------------------- */
/* The four data layouts compared in section 4 (Table 2: propagate and collide
 * on a 2160 x 8192 lattice), for timing those two kernels on each.  These
 * calls are stateless and separate from contexts: FP64 populations of an
 * lx x ly lattice, periodic in x and y, no halos, no padding, no walls.
 * Population l of site (x, y) is element
 *   AOS     (x ly + y) 37 + l              all populations of a site together
 *   SOA     (l lx + x) ly + y              one array per population
 *   CSOA    ((l lx + x) M + i) VL + k      y = k M + i, M = ly / VL
 *   CAOSOA  ((x M + i) 37 + l) VL + k      y = k M + i
 * CSOA and CAOSOA split each column into VL partitions of M rows; a cluster
 * of VL elements holds the rows at the same offset i in every partition, so
 * a hop in y moves whole clusters (the clustered layouts of section 4, with VL
 * the cluster width).  AOS and SOA take vl = 1; CSOA and CAOSOA take
 * vl = 1, 2, 4, ..., 64 with ly a multiple of vl and ly / vl >= 3.  lx, ly
 * >= 7 and lx ly <= 2^26.  All buffers are device pointers to
 * lbm_study_bytes() bytes (canonical arrays: FP64 [37][lx][ly], the same
 * size); calls enqueue on the given HIP stream (NULL: the null stream) and
 * return at once.  Errors: LBM_ERR_INVALID / LBM_ERR_SIZE for bad arguments
 * (nothing is launched), LBM_ERR_HIP for a failed launch; the message is
 * lbm_last_error(NULL). */
typedef enum { LBM_STUDY_AOS = 0, LBM_STUDY_SOA = 1, LBM_STUDY_CSOA = 2, LBM_STUDY_CAOSOA = 3 } lbm_study_layout;
/* Bytes of one population buffer in that layout; 0 if the arguments are invalid. */
size_t lbm_study_bytes(int layout, int vl, int lx, int ly);
/* canonical [37][lx][ly] -> layout buffer, and back. */
lbm_status lbm_study_pack(int layout, int vl, int lx, int ly, const double* canon, double* buf, void* hip_stream);
lbm_status lbm_study_unpack(int layout, int vl, int lx, int ly, const double* buf, double* canon, void* hip_stream);
/* propagate (eq. (4), pull form): dst_l(x, y) = src_l(x - e_x, y - e_y), both
 * coordinates periodic.  src and dst are distinct buffers of the layout. */
lbm_status lbm_study_propagate(int layout, int vl, int lx, int ly, const double* src, double* dst, void* hip_stream);
/* collide (eq. (2) with the equilibrium and gravity of lbm_collide), in place
 * on a buffer of the layout; tau > 0.5. */
lbm_status lbm_study_collide(int layout, int vl, int lx, int ly, double tau, double g_y, double* buf,
                             void* hip_stream);

/* ---- host cores, and host + GPU co-execution -------------------------------- */
/* Section 5 splits the lattice along x: m border columns on each side run on
 * the host's cores, the remaining lx - 2m columns on the accelerator, and the
 * two exchange three-column halos after every step.  Section 6 models the
 * time per step as max(T_acc, T_host) + T_swap with T_acc = (lx - 2m) ly tau_d
 * and T_host = 2m ly tau_h (one process: no inter-process term), which
 * is least where T_acc = T_host.  FP64 only; lattices are x-periodic, y as in
 * params.ybc; params.xmode / step_kind / layout / adjoint are ignored. */

/* One fused step (pull streaming, wall rule, collide) on host cores over a
 * whole x-periodic lattice in host memory, stored in the library's FP64
 * column layout (lbm_host_lattice_bytes per buffer; fill with lbm_host_pack).
 * These serve as the host part's building block and to time tau_h. */
size_t lbm_host_lattice_bytes(const lbm_params* p);               /* 0 if invalid */
/* canonical FP64 [37][lx][ly] (host) -> a buffer, and back; pack writes the
 * sites only (ghost rows and halo columns keep their contents). */
lbm_status lbm_host_pack(const lbm_params* p, const double* canon, double* buf);
lbm_status lbm_host_unpack(const lbm_params* p, const double* buf, double* canon);
/* n steps on nthreads host threads, alternating a -> b -> a ...: the state
 * after n steps is in a if n is even, else in b.  In y-periodic mode the
 * ghost rows of the source buffer are refreshed in place. */
lbm_status lbm_host_step(const lbm_params* p, double* a, double* b, int64_t n, int nthreads);

typedef struct lbm_hetero lbm_hetero;
/* Device workspace bytes of the GPU part for m border columns per side
 * (m = 0: the whole lattice on the GPU; else m >= 2 and lx - 2m >= 3);
 * 0 if invalid. */
size_t lbm_hetero_workspace_bytes(const lbm_params* p, int m);
/* Creates a co-executed lattice: the GPU part in the caller's device
 * workspace (256-byte aligned, lbm_hetero_workspace_bytes) on hip_stream, the
 * host part (2 m + 6 columns, two buffers) in pinned host memory the library
 * allocates, stepped by host_threads threads.  Errors as lbm_create. */
lbm_status lbm_hetero_create(const lbm_params* p, int m, int host_threads, void* dev_workspace, size_t bytes,
                             void* hip_stream, lbm_hetero** out);
void lbm_hetero_destroy(lbm_hetero* h);
/* Whole-lattice state as canonical FP64 [37][lx][ly] in host memory
 * (synchronous; allocates a temporary device copy of the GPU part). */
lbm_status lbm_hetero_set_pops(lbm_hetero* h, const double* host_canon);
lbm_status lbm_hetero_get_pops(lbm_hetero* h, double* host_canon);
/* n steps: per step, the GPU part's step is enqueued, the host part steps
 * meanwhile, then the halos are exchanged: each side packs what the other's
 * halo columns are read for (the populations that cross the seam, and the
 * wall rows of the rest), one copy each way on the stream, unpack.  Results
 * equal lbm_step on the whole lattice up to rounding order (the host part is
 * compiled separately). */
lbm_status lbm_hetero_step(lbm_hetero* h, int64_t n);
/* Per-step averages over the last lbm_hetero_step call, seconds:
 * out = {wall time, host step, GPU step (HIP events), halo exchange (HIP
 * events from the end of the GPU step through the GPU's unpack, plus the
 * host's unpack)}. */
lbm_status lbm_hetero_times(const lbm_hetero* h, double out[4]);
/* Message of the last error ("" if none); NULL: of lbm_hetero_create. */
const char* lbm_hetero_last_error(const lbm_hetero* h);

/* ---- misc ------------------------------------------------------------------ */

/* Waits for the context's stream; LBM_ERR_HIP if queued work failed. */
lbm_status lbm_sync(lbm_ctx* ctx);
/* Message of the last error on this context ("" if none); NULL ctx: last
 * error of lbm_create or of an lbm_study_* call on this thread. */
const char* lbm_last_error(const lbm_ctx* ctx);
/* Canonical population order (host arrays of 37). */
void lbm_velocity_table(int8_t ex[LBM_NPOP], int8_t ey[LBM_NPOP]);
/* Weights w_l and the scale c (host). */
void lbm_weights(double w[LBM_NPOP]);
double lbm_scale_c(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
