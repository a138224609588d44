/*
 * pplbm.h -- C ABI of the MI355X pseudo-potential D2Q9 lattice Boltzmann library.
 *
 * The method is that of Hu, Li & Uddin, "Force Method in a Pseudo-potential Lattice
 * Boltzmann Model" (arXiv:1412.5170).  One time step (lbm_step) is:
 *   rho = sum_a f_a (Eq. 3) -> psi(rho) from the K-rescaled Carnahan-Starling EOS
 *   (Eq. 29, Eq. 30, Eq. 7) -> interaction force F (Kupershtokh hybrid, Eq. 6; A = 0 is the
 *   Shan-Chen force of Eq. 4) -> forcing scheme (exact difference, Eq. 22; Guo, Eq. 23; Guo
 *   with Li's modified term, Eq. 31) -> BGK (Eq. 1) or MRT (Eq. 34-35) collision ->
 *   periodic streaming (Eq. 36).
 * By default one HIP kernel for gfx950 advances two time steps per pass over the populations
 * (lbm_set_launch: LBM_KERNEL_SWEEP2, temporal blocking in 64-lane wave strips, psi recomputed
 * from the populations in registers); an odd last step of an lbm_step call runs the one-step
 * sweep (LBM_KERNEL_SWEEP).  The two-pass step (a density/psi pass, then a fused force +
 * collide + stream pass) is kept as an alternative; every kernel gives bitwise the same state.
 *
 * Conventions
 *   - Every function returns LBM_OK (0) or a negative LBM_E* code; no exception crosses
 *     the ABI.  lbm_last_error() gives the text of the last failure on a handle.
 *   - Host arrays belong to the caller, are FP64, row-major with x fastest: index y*nx + x.
 *     A velocity array holds the pair (u_x, u_y) per node: index 2*(y*nx + x) + {0, 1}.
 *   - Device state: FP32 populations, population a of node (x, y) at
 *     y * row_stride + a * velocity_stride + x (lbm_strides): the nine rows of each y next to
 *     each other (LBM_LAYOUT_ROWS, the default: row_stride = 9 * pitch,
 *     velocity_stride = pitch) or nine planes one after the other (LBM_LAYOUT_PLANES:
 *     row_stride = pitch, velocity_stride = pitch * ny).  Two population buffers (read and write side of the step)
 *     and one psi plane (ny * pitch floats, node at y * pitch + x).  They belong to the
 *     handle unless lbm_attach supplied them; attached memory must outlive the handle.
 *   - Ordering of the nine velocities: e_0 = (0,0), e_1 = (1,0), e_2 = (0,1), e_3 = (-1,0),
 *     e_4 = (0,-1), e_5 = (1,1), e_6 = (-1,1), e_7 = (-1,-1), e_8 = (1,-1).
 *   - lbm_step and lbm_init are asynchronous on the handle's stream; lbm_read, lbm_stats and
 *     lbm_populations synchronise it.  One handle per stream; calls on one handle must not
 *     overlap.
 */
#ifndef PPLBM_H
#define PPLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)        /* invalid argument or unsupported combination            */
#define LBM_ENOMEM (-2)        /* host or device allocation failed                       */
#define LBM_EHIP (-3)          /* a HIP runtime call failed (text in lbm_last_error)     */
#define LBM_EUNSTABLE (-4)     /* non-finite state, psi^2 <= 0 or b rho / 4 >= 1         */
#define LBM_ENOTCONVERGED (-5) /* step cap reached before the convergence criterion     */
#define LBM_ESTATE (-6)        /* call out of order (e.g. step before init)              */

/* ---- physics parameters ----------------------------------------------------------------- */
enum { LBM_EOS_CARNAHAN_STARLING = 0, LBM_EOS_SBRAGAGLIA_SHAN = 1 };
enum { LBM_FORCE_EDM = 0, LBM_FORCE_GUO = 1, LBM_FORCE_GUO_LI = 2, LBM_FORCE_SC = 3 };
enum { LBM_COLL_BGK = 0, LBM_COLL_MRT = 1 };
/* Arithmetic precision of the kernels; the populations are stored in FP32 either way.  (The
 * value 0 is not used: FP32 arithmetic throughout misses 1e-5 after 100 steps.) */
enum { LBM_PREC_F64 = 1, LBM_PREC_MIXED = 2 };
/* Population layout in device memory (see lbm_strides). */
enum { LBM_LAYOUT_PLANES = 0, LBM_LAYOUT_ROWS = 1 };

/* Equation of state and effective density.
 * LBM_EOS_CARNAHAN_STARLING, Eq. 29-30: p = K (rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3
 *   - a rho^2), eta = b rho / 4, and psi from Eq. 7.  T is given relative to the exact critical
 *   temperature of Eq. 29 (dp/drho = d2p/drho2 = 0).  Paper values: a = 1, b = 4, R = 1
 *   (Sec. 4.1).  eps is ignored.
 * LBM_EOS_SBRAGAGLIA_SHAN, Eq. 33: psi = exp(-1/rho) for eps = 0, (rho / (1 + rho))^(1/eps)
 *   otherwise (eps > 0); the pressure is the one Eq. 7 implies, p0 = rho/3 + G psi^2 / 2, so the
 *   interaction strength G of lbm_force plays the role of temperature.  a, b, R, T_over_Tc and K
 *   are ignored.  With the hybrid force, A = -eps/2 makes the mechanical condition (Eq. 18)
 *   coincide with the Maxwell rule (Eq. 19). */
typedef struct {
    int kind;          /* LBM_EOS_CARNAHAN_STARLING or LBM_EOS_SBRAGAGLIA_SHAN */
    double a, b, R;
    double T_over_Tc;  /* reduced temperature, 0 < T/Tc < 1 for two phases */
    double K;          /* EOS rescale of Eq. 30, K > 0 */
    double eps;        /* Eq. 33 exponent (LBM_EOS_SBRAGAGLIA_SHAN), >= 0 */
} lbm_eos;

/* Interaction force and forcing scheme.
 *   F = -A sum_a w(|e_a|^2) U(x+e_a) e_a - (1-A) G psi(x) sum_a w(|e_a|^2) psi(x+e_a) e_a,
 *   U = G psi^2 / 2, w(1) = 1/3, w(2) = 1/12 (Eq. 4-6).  psi from p0 = rho/3 + G psi^2/2
 *   (Eq. 7), so G must be negative; the force does not depend on G except through Li's term.
 * scheme: LBM_FORCE_EDM (Eq. 22), LBM_FORCE_GUO (Eq. 23), LBM_FORCE_GUO_LI (Eq. 31: Guo's
 * term with v' = v + sigma F / ((tau - 1/2) psi^2); Eq. 32 gives eps = 16 sigma for G = -1),
 * LBM_FORCE_SC (Eq. 20-21: BGK towards f^eq(rho, u + tau F / rho), no source term; BGK only). */
typedef struct {
    int scheme;
    double A;      /* Kupershtokh hybrid weight; A = 0 is Eq. 4, A = 1 is Eq. 5 */
    double sigma;  /* Li's constant (LBM_FORCE_GUO_LI only) */
    double G;      /* interaction strength, < 0; the paper uses G = -1 (Sec. 4.3) */
} lbm_force;

/* Collision.  BGK: Eq. 1 with relaxation time tau.  MRT (Eq. 34-35): Lallemand-Luo moment
 * basis in the order (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy), Lambda =
 * diag(s_rho, s_e, s_eps, s_j, s_q, s_j, s_q, 1/tau, 1/tau); Guo's source in moment space;
 * with LBM_FORCE_GUO_LI, Li's extra stress 2 sigma F F / psi^2 enters each stress/energy
 * moment divided by (1/s_k - 1/2), which reduces exactly to Eq. 31 when every rate is 1/tau.
 * MRT requires LBM_FORCE_GUO or LBM_FORCE_GUO_LI. */
typedef struct {
    int kind;      /* LBM_COLL_BGK or LBM_COLL_MRT */
    double s_rho, s_e, s_eps, s_j, s_q;  /* MRT rates in (0, 2); ignored for BGK */
} lbm_collision;

/* Observables of Sec. 4 (Tables 3-7), reduced in FP64 in a fixed order (deterministic). */
typedef struct {
    double mass;        /* sum over nodes of rho */
    double rho_min, rho_max;
    double rho_probe_a; /* rho at probe node a (default: lattice centre) */
    double rho_probe_b; /* rho at probe node b (default: node (0, 0)) */
    double ratio;       /* max(rho_probe_a, rho_probe_b) / min(...) */
    double us_max;      /* max over nodes of |v|, v = u + F / (2 rho) */
    double dv_max;      /* max over nodes of |v - v_prev|_inf since the previous tracked call */
    long long step;     /* time steps taken since lbm_init */
    int nonfinite;      /* number of nodes with a non-finite rho or v, or undefined psi */
} lbm_stats_t;

typedef struct lbm lbm_t;

/* Create a handle for an nx x ny periodic lattice.  Validates the parameters (nx, ny >= 1,
 * tau > 1/2, G < 0, b > 0, K > 0, 0 < T/Tc, MRT only with Guo/Guo+Li, MRT rates in (0, 2))
 * and computes the absolute temperature; allocates no device memory.  *out receives the
 * handle (NULL on error). */
int lbm_create(int nx, int ny, const lbm_eos *eos, const lbm_force *force,
               const lbm_collision *collision, double tau, lbm_t **out);

/* Release the handle and any device memory it owns. */
void lbm_destroy(lbm_t *h);

/* Device layout the handle uses: row pitch in floats (>= nx), floats per population plane,
 * bytes of one population buffer (9 planes) and of the psi plane.  Any pointer may be NULL. */
int lbm_layout(const lbm_t *h, size_t *pitch_floats, size_t *plane_floats, size_t *f_bytes,
               size_t *psi_bytes);

/* Hand the handle caller-owned device memory (e.g. from torch): two population buffers of
 * f_bytes each and a psi plane of psi_bytes, all 256-byte aligned, plus the HIP stream
 * (hipStream_t, NULL for the default stream).  Replaces any memory the handle owned. */
int lbm_attach(lbm_t *h, void *f_a, void *f_b, void *psi, void *stream);

/* Select the stream later calls are issued on (hipStream_t, NULL = default stream). */
int lbm_set_stream(lbm_t *h, void *stream);

/* Arithmetic precision of the kernels.  The populations stay FP32 in memory either way, so
 * the memory traffic is the same.
 *   LBM_PREC_MIXED (default): FP32 arithmetic except the operations whose cancellation sets
 *     the accuracy of the FP32 state -- the density and momentum sums, the EOS and psi, the
 *     interaction force, u and v (u and F/(2 rho) nearly cancel in the light phase),
 *     w rho - f in the relaxation and the mass closure -- which run in FP64.
 *   LBM_PREC_F64: FP64 throughout.
 * Both keep the state within 1e-5 of an FP64 run after 100 steps (FP32 arithmetic throughout
 * measured 1.1e-5 to 1.9e-5 and is rejected with LBM_EINVAL). */
int lbm_set_precision(lbm_t *h, int precision);

/* Population layout (LBM_LAYOUT_PLANES or LBM_LAYOUT_ROWS); only before lbm_init or
 * lbm_set_populations.  Results do not depend on the layout. */
int lbm_set_layout(lbm_t *h, int layout);

/* Strides (in floats) of the population buffers: node (x, y), velocity a at
 * y * row_stride + a * velocity_stride + x. */
int lbm_strides(const lbm_t *h, size_t *row_stride, size_t *velocity_stride);

/* Kernel shape of lbm_step.  Every choice computes bitwise the same result.  The default is
 * the two-step sweep (LBM_KERNEL_SWEEP2, tx = 256, LBM_LAUNCH_XCD_ORDER) on every lattice,
 * with S = ceil(nx / 58) strips: ty = 16 where S * ceil(ny / 16) >= 8192 (from about 3000^2), else
 * ty = 24 where S * ceil(ny / 24) >= 3072 (about 2048^2), else the ty between 6 and 24 that
 * gives about 3200 waves; where that is 6 (lattices up to about 1024^2, too small to fill the
 * GPU), tx = 64 and the ty in 1..12 that minimises (ty + 4) max(1.5, ceil(W / 1024)), W =
 * S * ceil(ny / ty) waves: rows per wave times waves per SIMD.  The odd last step of an
 * lbm_step call runs the one-step sweep with
 * tx = 512, ty = 8, two rows of loads in flight and LBM_LAUNCH_XCD_ORDER, narrowed (tx, then
 * ty) on small lattices until the launch has about 1024 workgroups.
 *   LBM_KERNEL_TWO_PASS: the density/psi pass writes psi, then the fused pass
 *     reads it; (tx, ty) = threads per workgroup of the fused pass (tx a multiple of 64,
 *     tx * ty <= 1024).  116 bytes of memory traffic per node and step.
 *   LBM_KERNEL_SWEEP: one kernel per step; a workgroup of tx threads (multiple of 64, <= 512)
 *     sweeps a strip of tx columns over segments of ty rows, computing psi from the
 *     populations as it loads them, so each population is read once: 72 bytes per node and
 *     step plus the strip and segment edges.  Addresses the populations through 32-bit
 *     buffer offsets: from the buffer's start while it is below 4 GiB, else from each row's
 *     start (about 3 % slower), which needs LBM_LAYOUT_ROWS -- a planes-layout lattice beyond
 *     4 GiB takes the two-pass step (LBM_EINVAL for the sweep; lbm_set_layout switches it).
 *     The batch's lattices must stay below 4 GiB each.
 *   LBM_KERNEL_SWEEP2: two time steps per launch (temporal blocking): each 64-lane wave sweeps
 *     a strip of 58 output columns over segments of ty rows, computing step t on its 64
 *     columns and step t+1 two rows behind; lanes exchange x-neighbours by DPP shifts, so no
 *     LDS or barrier is used, and only step t+1 is written: 72 bytes per node per two steps
 *     plus the strip and segment overlaps.  tx = threads per workgroup (independent waves,
 *     multiple of 64, <= 256).  An odd last step of lbm_step runs the one-step sweep.  Beyond
 *     4 GiB of populations it addresses rows like the one-step sweep (rows layout only).
 * flags: LBM_LAUNCH_NONTEMPORAL (non-temporal stores of the new populations),
 *        LBM_LAUNCH_XCD_ORDER (consecutive tiles on the same XCD; both sweeps),
 *        LBM_LAUNCH_SHALLOW (sweep only: load one row ahead instead of two; fewer registers). */
enum { LBM_KERNEL_TWO_PASS = 0, LBM_KERNEL_SWEEP = 1, LBM_KERNEL_SWEEP2 = 2 };
#define LBM_LAUNCH_NONTEMPORAL 1
#define LBM_LAUNCH_XCD_ORDER 2
#define LBM_LAUNCH_SHALLOW 4
#define LBM_LAUNCH_SERIAL_KINDS 8 /* batch only: see lbm_batch_set_launch */
#define LBM_LAUNCH_TWO_STEP 16    /* batch only: see lbm_batch_set_launch */
int lbm_set_launch(lbm_t *h, int kernel, int tx, int ty, int flags);
int lbm_get_launch(const lbm_t *h, int *kernel, int *tx, int *ty, int *flags);

/* Shorthand for lbm_set_launch(h, LBM_KERNEL_TWO_PASS, tx, ty, current flags). */
int lbm_set_tile(lbm_t *h, int tx, int ty);

/* Probe nodes reported by lbm_stats (defaults: a = (nx/2, ny/2), b = (0, 0)). */
int lbm_set_probes(lbm_t *h, int xa, int ya, int xb, int yb);

/* Initial state f_a = f^eq_a(rho0, u0) (Eq. 2) from host FP64 fields; u0 may be NULL (rest).
 * Allocates the device buffers on first use if none were attached.  Resets the step count. */
int lbm_init(lbm_t *h, const double *rho0, const double *u0);

/* Advance n >= 0 time steps (Sec. 2-4; Eq. 1 or Eq. 34-36), asynchronously. */
int lbm_step(lbm_t *h, int n);

/* Density (Eq. 3) and actual fluid velocity v = u + F/(2 rho) (Sec. 3.2) of the current
 * state into host FP64 arrays (either may be NULL).  Synchronises the stream. */
int lbm_read(lbm_t *h, double *rho, double *u);

/* Current populations as FP32 host array [9][ny][nx] (velocity order above). Synchronises. */
int lbm_populations(lbm_t *h, float *f);

/* Replace the populations from a host FP32 array [9][ny][nx]; keeps the step count. */
int lbm_set_populations(lbm_t *h, const float *f);

/* Checkpoint: lbm_save writes the populations (FP32), the step count and the parameter structs
 * to `path`; lbm_load restores them into a handle created with the same size and parameters
 * (LBM_EINVAL otherwise, or for a file this library did not write).  Both synchronise.  The
 * file holds native-endian binary data. */
int lbm_save(lbm_t *h, const char *path);
int lbm_load(lbm_t *h, const char *path);

/* FP64 observables of the current state.  track_dv != 0 also compares v with the velocity
 * stored by the previous tracked call (dv_max; 0 on the first) and stores the current one.
 * Returns LBM_EUNSTABLE (with *out filled) when a node is non-finite. Synchronises. */
int lbm_stats(lbm_t *h, int track_dv, lbm_stats_t *out);

/* Allocation-free variant of lbm_stats, for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): lbm_stats with track_dv = 0 and without the
 * reduction buffers lbm_stats allocates on first use.  It runs the same kernels on the same
 * block partition, so it reports the same values bit for bit (dv_max = 0: no velocity history).
 * The reduction's partial results and result vector live in a fixed device array of the
 * library, 2048 x 6 + 8 doubles (96.06 KiB) on each GPU it runs on, held until the process
 * ends; every lattice fits (the reduction uses at most 2048 blocks), and a larger need would
 * return LBM_EINVAL.  All calls on one GPU share that array; each call writes everything it
 * reads, so nothing needs clearing, but calls that overlap on one GPU (two threads, two
 * streams) race on it and must be serialised by the caller.  The handle's GPU must be the
 * current device; needs lbm_init or lbm_set_populations first (LBM_ESTATE).  Calls no
 * allocator; synchronises the handle's stream (so it cannot be recorded into a graph).
 * Returns LBM_EUNSTABLE (with *out filled) when a node is non-finite. */
int lbm_stats_noalloc(lbm_t *h, lbm_stats_t *out);

/* Autotuner: times trial_steps steps (rounded up to even) of the one-pass sweep for strip widths
 * tx in {64, 128, 256, 512}, segment heights ty in {4, 8, 16, 32, 64} and the flag sets
 * XCD|SHALLOW, SHALLOW, XCD, XCD|SHALLOW|NONTEMPORAL, and of the two-step sweep for tx in
 * {64, 128, 256}, ty in {1, 2, 3, 4, 6, 8, 12, 16, 24, 32} and the flags XCD or none; a
 * planes-layout lattice beyond 4 GiB, where neither sweep runs, tries the two-pass step for tx in
 * {64, 128, 256} and ty in {2, 4, 8} (tx * ty <= 1024) with LBM_LAUNCH_XCD_ORDER.  Shapes are
 * bitwise equivalent, so only speed differs.  Keeps the fastest and applies it with
 * lbm_set_launch.  Runs on the current state, which it saves and
 * restores (populations and step count), so the simulation resumes exactly where it was.
 * cache_path (may be NULL): JSON lines keyed by device, size, scheme, collision, precision and
 * layout; a hit applies the cached launch without trials (*ms_out = -1).  *ms_out (may be
 * NULL): the best time per step in ms.  Needs lbm_init first.  Synchronises. */
int lbm_autotune(lbm_t *h, const char *cache_path, int trial_steps, double *ms_out);

/* Kernel timing with HIP events recorded on the handle's stream while enabled: the two-pass
 * step around each of its two launches, every step; the one-pass sweep around each lbm_step
 * call's n back-to-back launches (an event between launches would cost ~5 % of the step).
 * lbm_timing returns the summed milliseconds of the density/psi pass and of the fused pass
 * (with the sweep: ~0 and the sweep kernels) and the number of steps timed, then resets them.
 * While enabled, pending events are folded into the sums every 1024 timed calls or steps (one
 * host synchronisation), so memory stays bounded. */
int lbm_timing_enable(lbm_t *h, int enable);
int lbm_timing(lbm_t *h, double *psi_ms, double *fused_ms, long long *steps);

/* ---- batched sweep ---------------------------------------------------------------------------
 * Many independent periodic lattices, each with its own size, EOS temperature and rescale,
 * force, collision and relaxation time (the parameter sweeps of Sec. 4 as one job), advanced
 * together: by default one launch per kernel kind advances two time steps, one wave per tile
 * of a shared device list of tiles (a 58-column strip x a segment of rows of one lattice; one
 * step per launch walks a list of tx-column strips with persistent workgroups instead); blocks
 * of steps are captured in a hipGraph and replayed; lattices that converge or go unstable are
 * dropped from the tile lists in device memory between replays (the graph is captured again
 * when a kind's tile count changes).  Per-node arithmetic is the single-lattice sweep's (mixed precision,
 * row-interleaved layout), so each lattice evolves bitwise as it would alone.  The batch owns
 * its device memory and a HIP stream of its own (default priority). */
typedef struct lbm_batch lbm_batch_t;

/* count lattices; arrays of count entries.  Validation as lbm_create. */
int lbm_batch_create(int count, const int *nx, const int *ny, const lbm_eos *eos,
                     const lbm_force *force, const lbm_collision *collision, const double *tau,
                     lbm_batch_t **out);
void lbm_batch_destroy(lbm_batch_t *b);

/* Launch of the batch's one-step kernel: tx threads per workgroup (multiple of 64, <= 512),
 * `groups` persistent workgroups per kernel kind (0: one per tile up to 2048; rounded down to a
 * multiple of 8, each XCD walking its own eighth of the tile list); flags
 * LBM_LAUNCH_NONTEMPORAL | LBM_LAUNCH_SHALLOW | LBM_LAUNCH_SERIAL_KINDS | LBM_LAUNCH_TWO_STEP.
 * A kernel kind is a forcing scheme: exact difference and Shan-Chen (BGK), Guo and Guo + Li
 * (BGK and MRT lattices share one kernel, the collision being computed in moment space).  The
 * captured graph holds one chain of launches, kind after kind, on the batch's stream
 * (LBM_LAUNCH_SERIAL_KINDS is accepted and is the only behaviour).  LBM_LAUNCH_TWO_STEP
 * advances two steps per launch with the single lattice's two-step sweep: one 64-lane wave per
 * tile (a strip of 58 output columns over a segment of 1 to 24 rows, the height chosen at every
 * change of the active set by the single lattice's rule applied to the active lattices' total
 * wave count); with n = 2 mod 4 steps the last two are one-step launches.  Results are bitwise
 * the same in every case.  Default: tx = 256, groups = 0, flags = LBM_LAUNCH_TWO_STEP. */
int lbm_batch_set_launch(lbm_batch_t *b, int tx, int groups, int flags);

/* Segment height (rows per tile) of lattice i; 0 (the default) is automatic: every time the
 * tile list is rebuilt (lattices activated or dropped), the automatic lattices share one height,
 * halved from 32 down to 4 rows until the active tiles number about 4096, so the lattices still
 * running when most have converged spread over the whole GPU.  The autotuner sets it per size
 * class.  Results do not depend on it (bitwise). */
int lbm_batch_set_segment(lbm_batch_t *b, int i, int rows);

/* f = f^eq(rho0, u0) for lattice i (host FP64 [ny][nx], u0 [ny][nx][2] or NULL); makes it
 * active and resets its step count. */
int lbm_batch_init(lbm_batch_t *b, int i, const double *rho0, const double *u0);

/* Lattice i at physical rest with density rho0 (host FP64 [ny][nx]): f = f^eq(rho0, u) with
 * u = -F / (2 rho0), F the interaction force of rho0 (Eq. 6 with psi of Eq. 7), so that the
 * fluid velocity v = u + F / (2 rho) (Sec. 3) is zero everywhere.  A bare f^eq(rho0, 0) start
 * (lbm_batch_init with u0 = NULL) gives every interface node the velocity F / (2 rho), an
 * impulse whose ringing sets the time to equilibrium even from an exact equilibrium density.
 * Makes the lattice active and resets its step count.  Synchronises. */
int lbm_batch_init_rest(lbm_batch_t *b, int i, const double *rho0);

/* The plain start of the droplet sweeps: rho = (rho_in + rho_out)/2 - (rho_in - rho_out)/2
 * tanh(2 (r - R) / W), r the distance from (nx/2, ny/2), with the Maxwell densities of the
 * lattice's EOS (lbm_coexistence) -- liquid inside for droplet != 0, gas inside (a bubble)
 * otherwise -- set at physical rest as in lbm_batch_init_rest.  Synchronises. */
int lbm_batch_init_tanh(lbm_batch_t *b, int i, double R, double W, int droplet);

/* Warm start of lattice i from a radial profile (the learned initial state): log_rho holds 64
 * host values of log rho at the radii r_k = r0 + k dr (k = 0..63, dr > 0), r the distance from
 * (nx/2, ny/2); rho(x, y) = exp(L(r - shift)) with L the piecewise-linear interpolant, held at
 * the first value below r0 and at the last beyond r0 + 63 dr; set at physical rest as in
 * lbm_batch_init_rest.  mass > 0: the shift (within +- half the lattice diagonal) whose total
 * density sum equals `mass` (relative 1e-13; bisection) -- in a periodic box the mass fixes the
 * equilibrium, so a warm start must carry the mass of the state it replaces; mass <= 0: shift
 * 0.  *shift_out (may be NULL) receives the shift.  LBM_EINVAL if a value is not finite or no
 * shift reaches the mass; LBM_EUNSTABLE if the density leaves (0, 4/b) (Carnahan-Starling).
 * Makes the lattice active and resets its step count.  Synchronises. */
int lbm_batch_init_profile(lbm_batch_t *b, int i, const double *log_rho, double r0, double dr,
                           double mass, double *shift_out);

/* Autotuner for the batch: times trial_steps (even) steps of every lattice for strip widths
 * tx in {64, 128, 256, 512} with and without LBM_LAUNCH_SHALLOW, then, per size class (lattices whose
 * longer side rounds up to the same power of two), segment heights {8, 16, 32, 64}; keeps the
 * fastest and applies it.  Needs every lattice initialised; saves and restores the populations,
 * step counts and activity flags, so the batch resumes exactly where it was.  cache_path (may be
 * NULL): JSON lines keyed by device and the multiset of (size, scheme, collision); a hit
 * applies the cached choice without trials (*ms_out = -1).  *ms_out (may be NULL): the best
 * time per step in ms.  Synchronises. */
int lbm_batch_autotune(lbm_batch_t *b, const char *cache_path, int trial_steps, double *ms_out);

/* Include (1) or exclude (0) an initialised lattice from stepping. */
int lbm_batch_set_active(lbm_batch_t *b, int i, int active);

/* n (even) steps of every active lattice, asynchronously on the batch stream. */
int lbm_batch_step(lbm_batch_t *b, int n);

/* FP64 observables of every active lattice into out[i] (out has count entries); track_dv as in
 * lbm_stats.  Synchronises.  LBM_EUNSTABLE if any lattice has non-finite nodes. */
int lbm_batch_stats(lbm_batch_t *b, int track_dv, lbm_stats_t *out);

/* Step every active lattice until it has converged (status 0) -- max_x |v(t) - v(t - k)|_inf / k
 * < tol and, if tol_rho > 0, the relative change of both probe densities over the last k steps,
 * divided by k, < tol_rho (k = check_every, even) -- or a node goes non-finite (LBM_EUNSTABLE)
 * or max_steps is reached (LBM_ENOTCONVERGED).  steps_out / status_out: count entries (either
 * may be NULL).  Lattices already inactive keep status LBM_ESTATE. */
int lbm_batch_run(lbm_batch_t *b, double tol, double tol_rho, int check_every,
                  long long max_steps, long long *steps_out, int *status_out);

/* rho and v of lattice i (as lbm_read); its populations as FP32 [9][ny][nx]. */
int lbm_batch_read(lbm_batch_t *b, int i, double *rho, double *u);
int lbm_batch_populations(lbm_batch_t *b, int i, float *f);

/* Steps taken by lattice i (-1 for a bad index); wait for the batch stream; error text. */
long long lbm_batch_steps(const lbm_batch_t *b, int i);
int lbm_batch_sync(lbm_batch_t *b);
const char *lbm_batch_last_error(const lbm_batch_t *b);

/* ---- learned warm start: multilayer perceptron ---------------------------------------------
 * Dense layers dims[0] -> dims[1] -> ... -> dims[nlayers], tanh on every hidden layer, linear
 * output, FP32 on the GPU; trained with mean-squared error and Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8).  Parameters are one flat FP32 vector: for each layer l, W_l (row-major
 * [dims[l+1]][dims[l]]) then b_l.  x, y, target, dy and grad are device pointers (row-major
 * [batch][dim]); `stream` is a hipStream_t (NULL = default).  Used to predict a droplet's
 * radial density profile from (T/Tc, tau, R, K) as the initial state of the batched sweep. */
typedef struct lbm_mlp lbm_mlp_t;
int lbm_mlp_create(int nlayers, const int *dims, lbm_mlp_t **out);
void lbm_mlp_destroy(lbm_mlp_t *n);
size_t lbm_mlp_param_count(const lbm_mlp_t *n);
/* Host FP32 parameter vector in / out; setting it also resets the Adam state. */
int lbm_mlp_set_params(lbm_mlp_t *n, const float *host_params);
int lbm_mlp_get_params(lbm_mlp_t *n, float *host_params);
/* y = net(x). */
int lbm_mlp_forward(lbm_mlp_t *n, const float *x, int batch, float *y, void *stream);
/* grad = d(sum_b sum_o dy[b][o] y[b][o]) / d(parameters) at x (one forward + backward pass). */
int lbm_mlp_gradient(lbm_mlp_t *n, const float *x, const float *dy, int batch, float *grad,
                     void *stream);
/* One Adam step on the mean-squared error mean((net(x) - target)^2) with learning rate lr;
 * *loss_out (may be NULL) receives the loss before the step (synchronises when given). */
int lbm_mlp_train_step(lbm_mlp_t *n, const float *x, const float *target, int batch, float lr,
                       float *loss_out, void *stream);
const char *lbm_mlp_last_error(const lbm_mlp_t *n);

/* ---- EOS helpers (host only) -------------------------------------------------------------- */

/* Exact critical point of Eq. 29 (independent of K): dp/drho = d2p/drho2 = 0. */
int lbm_eos_critical(const lbm_eos *eos, double *rho_c, double *T_c, double *p_c);

/* Maxwell equal-area coexistence densities (Eq. 19) at eos->T_over_Tc; independent of K
 * (Sec. 4.1).  Solved as equal pressure and equal chemical potential of the two phases with
 * the Carnahan-Starling free energy.  Carnahan-Starling only (LBM_EINVAL otherwise). */
int lbm_eos_maxwell(const lbm_eos *eos, double *rho_g, double *rho_l);

/* Coexistence densities of a flat interface for either EOS kind (host only).
 *   LBM_COEX_MAXWELL:    Eq. 19, p0(rho_g) = p0(rho_l) = p_c and the integral of
 *                        (p_c - p0) / rho^2 over [rho_g, rho_l] vanishes;
 *   LBM_COEX_MECHANICAL: Eq. 18, the same with the weight psi' / psi^(1 + eps_mech), psi from
 *                        Eq. 7 (Carnahan-Starling, where G only scales psi) or Eq. 33.
 * eps_mech is the exponent of Eq. 18 (eps = -2A for the hybrid force of Eq. 6, Table 1;
 * Eq. 32 for Li's model); ignored by LBM_COEX_MAXWELL.  For the Eq. 33 kind p0 = rho/3 +
 * G psi^2 / 2, so force->G matters.  Spinodals by a scan of dp0/drho and bisection, branch
 * densities by bisection, the integral by composite Gauss-Legendre in ln(rho), p_c by
 * bisection.  LBM_EINVAL for bad arguments or when p0 has no van der Waals loop. */
enum { LBM_COEX_MAXWELL = 0, LBM_COEX_MECHANICAL = 1 };

/* Bulk pressure p0(rho) (host): Eq. 30 for the Carnahan-Starling kind, rho/3 + G psi^2 / 2 with
 * psi of Eq. 33 for the other (Eq. 7).  Used for Laplace's law on bubbles (Table 3). */
int lbm_eos_pressure(const lbm_eos *eos, const lbm_force *force, double rho, double *p);
int lbm_coexistence(const lbm_eos *eos, const lbm_force *force, int rule, double eps_mech,
                    double *rho_g, double *rho_l);

/* ---- error text ----------------------------------------------------------------------------- */
const char *lbm_strerror(int code);
const char *lbm_last_error(const lbm_t *h);

/* ---- measurement aid ----------------------------------------------------------------------- */
/* Copy n floats src -> dst (device pointers) with a plain streaming kernel on `stream`.
 * Its HBM counters give the scale factor for the library's own kernels' counters. */
int lbm_copy_f32(float *dst, const float *src, size_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PPLBM_H */
