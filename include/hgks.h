/*
 * hgks.h - C ABI of the MI355X (gfx950) high-order gas-kinetic scheme hot path.
 *
 * The library advances cell-averaged conserved variables
 * Q = (rho, rho U, rho V, rho W, rho E) on a 3D structured box grid with the
 * high-order gas-kinetic scheme of arXiv 2207.01173, Sec. 2:
 *   - fifth-order WENO-Z reconstruction, dimension by dimension, of values and
 *     normal/tangential slopes at the 2x2 Gauss points of every cell face;
 *   - the time-dependent BGK gas distribution at each Gauss point, Eq. (flux),
 *     with the equilibrium from the compatibility condition and tau = mu/p;
 *   - the time-integrated flux over [0, dt] and [0, dt/2], giving the flux and
 *     its time derivative, Eq. (expansion-1);
 *   - the two-stage fourth-order update, Eq. (two-stage);
 *   - ghost cells synthesised on the fly (periodic, or an isothermal no-slip
 *     wall on the y axis), the CFL time step, and volume statistics
 *     (kinetic energy and viscous dissipation, Sec. 4.1).
 *
 * Memory: every device pointer is caller-owned (allocated by the caller, e.g.
 * through PyTorch).  The state array q_dev is float64 SoA [5][nz][ny][nx],
 * x fastest, and always holds the latest state once the stream has drained.
 * The workspace is an opaque device buffer of hgks_workspace_size() bytes,
 * 256-byte aligned.  The library allocates only its host-side context (and
 * nothing at all in hgks_residual_static).
 *
 * Streams: all device work of a context is enqueued on the hipStream_t given
 * to hgks_init (passed as void*).  hgks_step is asynchronous; hgks_stats,
 * hgks_dt and hgks_residual synchronise that stream before returning.
 *
 * Errors: functions return an hgks_status.  Argument and configuration errors
 * are detected before any device work (HGKS_E_INVALID).  A HIP runtime error
 * returns HGKS_E_DEVICE; the detail text is available from hgks_last_error().
 * A non-finite or non-positive density/pressure found by hgks_stats is latched
 * and returned by the following hgks_step (HGKS_E_NONFINITE /
 * HGKS_E_NEGATIVE_STATE) without advancing.
 *
 * Threads: a context must not be used from two threads at once; distinct
 * contexts are independent.
 */
#ifndef HGKS_H
#define HGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HGKS_ABI_VERSION 2

/* hgks_config.flags bit 0: constant streamwise mass flux (Sec. 4.2, where a
 * constant streamwise momentum flux determines the external force).  The
 * target is the volume mean of rho U of the state given to hgks_init; after
 * each step the x body force becomes f - (2 e^{n+1} - e^n) / (rho_b dt), e the
 * deviation of the step's mean rho U from the target, rho_b the initial mean
 * density; body_force[0] is the starting force.  Per instance, in a
 * single-instance context or as a batch member alike. */
#define HGKS_FLAG_CONSTANT_MASS_FLUX 1

typedef struct hgks_ctx_s* hgks_ctx;

typedef enum {
  HGKS_OK = 0,
  HGKS_E_INVALID = 1,        /* bad argument, configuration or workspace size */
  HGKS_E_NOMEM = 2,          /* host allocation failed */
  HGKS_E_DEVICE = 3,         /* HIP runtime error (see hgks_last_error) */
  HGKS_E_NONFINITE = 4,      /* the state holds NaN or Inf */
  HGKS_E_NEGATIVE_STATE = 5, /* density or pressure <= 0 somewhere */
  HGKS_E_UNSUPPORTED = 6     /* valid request the library does not provide */
} hgks_status;

enum { HGKS_BC_PERIODIC = 0, HGKS_BC_ISOTHERMAL_WALL = 1 }; /* wall: y axis only */
/* Precision of a context.  FP64: everything in FP64.  MIXED: reconstruction
 * and Gauss-point flux in FP32 on deviations from the initial state's volume
 * mean, state, update and reductions FP64.  FP32: additionally the state, Q*
 * and the S2O4 accumulator in FP32 (an FP32 working copy; hgks_step reads the
 * caller's FP64 state when it starts and writes it back when it ends), the
 * face fluxes and reductions staying FP64; the whole-code FP32 point of the
 * paper's precision comparison (Sec. 4.2).  Batched contexts: FP64 or MIXED. */
enum { HGKS_FP64 = 0, HGKS_MIXED = 1, HGKS_FP32 = 2 };

typedef struct {
  int32_t abi_version;   /* must equal HGKS_ABI_VERSION */
  int32_t n[3];          /* interior cells nx, ny, nz; each >= 4 */
  double lo[3], hi[3];   /* physical box; y walls (if any) at lo[1], hi[1] */
  int32_t bc[3];         /* HGKS_BC_* per axis; a wall only on axis 1 */
  double y_stretch;      /* tanh stretching b of the y axis (Sec. 4.2 map); 0: uniform */
  double gamma;          /* specific heat ratio, 1 < gamma <= 5/3 */
  double prandtl;        /* Prandtl number (heat-flux correction when != 1) */
  double mu_ref, T_ref, mu_exp; /* mu = mu_ref (T/T_ref)^mu_exp, T = p/rho */
  double T_wall;         /* isothermal wall temperature (p/rho units) */
  double body_force[3];  /* constant acceleration (source in L) */
  double cfl;            /* CFL number of the time-step rule when dt is not fixed */
  double rho_ref;        /* rho0 of the statistics normalisation (> 0) */
  int32_t precision;     /* HGKS_FP64, HGKS_MIXED or HGKS_FP32 */
  int32_t flags;         /* 0 or HGKS_FLAG_CONSTANT_MASS_FLUX */
} hgks_config;

typedef struct {
  double t;              /* simulated time since hgks_init's t0 origin */
  double dt_last;        /* last time step used */
  int64_t steps;         /* steps taken since hgks_init */
  double Ek;             /* (1/(rho0 Omega)) int rho |U|^2 / 2 */
  double eps_sol;        /* (mu_ref/(rho0 Omega)) int omega . omega */
  double eps_dil;        /* (4/3)(mu_ref/(rho0 Omega)) int (div U)^2 */
  double eps_com;        /* eps_sol + eps_dil (Sec. 4.1 total viscous dissipation) */
  double total[5];       /* int Q dV */
  double max_abs[5];     /* max |Q| per component */
  double min_p, min_rho; /* minima of pressure and density */
  int32_t nonfinite;     /* 1 if any NaN/Inf was found */
  int32_t pad_;
  double body_force_x;   /* x body force in effect (the controller's with the mass-flux flag) */
} hgks_stats_t;

/* Workspace bytes for a configuration.  Errors: HGKS_E_INVALID, also for a
 * grid too large for the kernels' 32-bit offsets into the face buffer: for
 * each face direction, with (e_x, e_y, e_z) that direction's face extents
 * (n along a periodic normal, whose face n is face 0, n + 1 along a wall
 * normal, n elsewhere, plus 2 ghost faces on each side of a wall axis when it
 * is the second tangential one) and pitch = e_x rounded up to 32,
 * 16 x pitch x e_y x (e_z + 1) bytes must stay below 2^32 (a periodic 640^3
 * grid is accepted, 641^3 is not). */
hgks_status hgks_workspace_size(const hgks_config* cfg, size_t* bytes);

/* Create a context over caller-owned memory: q_dev (state, in/out), ws_dev
 * (>= hgks_workspace_size bytes, 256-byte aligned) and a HIP stream (NULL:
 * the default stream).  t0 is the initial simulated time.  Enqueues the
 * geometry upload and the first wave-speed reduction on the stream. */
hgks_status hgks_init(const hgks_config* cfg, double* q_dev, void* ws_dev, size_t ws_bytes,
                      void* hip_stream, double t0, hgks_ctx* out);

/* Advance nsteps S2O4 steps (Eq. (two-stage)).  dt_fixed > 0 uses that time
 * step; dt_fixed <= 0 takes dt = cfl / max_cells max_d (|U_d| + c) / h_d from
 * the state at the start of each step.  Asynchronous.  On a created stream
 * one step is captured in a HIP graph at the first call and replayed nsteps
 * times (one launch per step; the time-step rule is a device value, so the
 * graph serves every dt_fixed); on the default stream, with profiling
 * enabled, or on a stream the caller is capturing, the kernels are launched
 * one by one.  Both give bit-identical results. */
hgks_status hgks_step(hgks_ctx ctx, int32_t nsteps, double dt_fixed);

/* Statistics of the current state (synchronises the stream). */
hgks_status hgks_stats(hgks_ctx ctx, hgks_stats_t* out);

/* CFL time step of the current state (synchronises the stream). */
hgks_status hgks_dt(hgks_ctx ctx, double* dt_out);

/* L(Q) and dL/dt (Eq. (semi2) and its time derivative) of an arbitrary state
 * q_dev (same layout as the context's state) with flux windows [0, dt] and
 * [0, dt/2]; outputs L_dev, dL_dev in the same layout.  Uses the context's
 * workspace; synchronises the stream. */
hgks_status hgks_residual(hgks_ctx ctx, const double* q_dev, double dt, double* L_dev, double* dL_dev);

/* hgks_residual without a context or a workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): computes on hip_stream (NULL: the default
 * stream; it must belong to the current HIP device) the same L(Q) and dL/dt of
 * q_dev, a float64 [5][nz][ny][nx] state of configuration cfg, with flux
 * windows [0, dt] and [0, dt/2], into L_dev and dL_dev (same layout; all three
 * caller-owned).  The body force is cfg->body_force; the mixed and FP32
 * precisions reconstruct on deviations from the volume mean of q_dev (what
 * hgks_residual does on a context initialised with q_dev).
 * Memory: the library allocates nothing, host or device.  Its face buffers,
 * metric arrays and scalars live in one static device array of
 * HGKS_STATIC_SCRATCH_BYTES bytes per GPU, which each GPU the library runs on
 * holds from the library's load until the process ends; every call on a GPU
 * reuses that GPU's array.  Calls that overlap on one GPU (two streams, or two
 * threads) race on it and give undefined results; calls on one stream are
 * ordered and safe.
 * Asynchronous: returns after enqueueing (no synchronisation), so it can be
 * captured in a HIP graph.
 * Errors (the detail text of the calling thread's last failure:
 * hgks_last_error(NULL)): HGKS_E_INVALID for an invalid configuration, a null
 * or misaligned pointer or dt not positive and finite; HGKS_E_UNSUPPORTED for
 * a grid whose face buffers exceed the static array (a periodic cube of up to
 * 36^3 cells fits in FP64, 34^3 with walls on y; 44^3 and 43^3 with the FP32
 * face data of the mixed and FP32 precisions); HGKS_E_DEVICE for a HIP
 * error. */
#define HGKS_STATIC_SCRATCH_BYTES (64u << 20)
hgks_status hgks_residual_static(const hgks_config* cfg, const double* q_dev, double dt, double* L_dev,
                                 double* dL_dev, void* hip_stream);

/* Kernel timing for benchmarks, with HIP events recorded on the context's
 * stream.  enable != 0: every kernel launch made by hgks_step is bracketed by
 * a pair of events.  hgks_profile_read synchronises the stream and returns,
 * per kernel class, the summed milliseconds and launch counts since the last
 * read, then resets them.  Classes: 0 reconstruction (normal and first
 * tangential sweep), 1 flux (second tangential sweep, Gauss-point flux,
 * face assembly), 2 cell update, 3 other.  Errors: HGKS_E_INVALID,
 * HGKS_E_DEVICE. */
#define HGKS_PROFILE_CLASSES 4
hgks_status hgks_profile(hgks_ctx ctx, int32_t enable);
hgks_status hgks_profile_read(hgks_ctx ctx, double ms[HGKS_PROFILE_CLASSES], int64_t launches[HGKS_PROFILE_CLASSES]);

/* Measurement aid for roofline figures, not a step of the method: the FP64
 * FMA rate this GPU sustains now.  Launches blocks x 256 threads on hip_stream
 * (NULL: the default stream); each thread runs 8 independent chains of iters
 * dependent FP64 FMAs (16 iters operations per thread) and writes the sum of
 * its chains to out_dev[block * 256 + thread] (caller-owned device memory of
 * blocks * 256 doubles).  Asynchronous; time it with events on the same
 * stream.  Errors: HGKS_E_INVALID (null out_dev, blocks or iters not
 * positive), HGKS_E_DEVICE. */
hgks_status hgks_fma_probe(double* out_dev, int32_t blocks, int32_t iters, void* hip_stream);

/* ---- Batched ensemble ----------------------------------------------------
 * Many independent instances (each its own grid size, gas and state) advanced
 * together: every phase of a step is one launch over the concatenated tile
 * work list of all instances (or of a group of consecutive instances whose
 * reconstruction buffers fit a cache budget; the autotuner picks the budget and
 * the flux tile width at init, timing the candidates on the ensemble's own
 * state), each S2O4 step is captured once in a HIP graph and replayed, and
 * each instance takes its own CFL time step.  Instance i's state q_devs[i] has
 * the single-instance layout, and each instance's arithmetic is that of a
 * single-instance run (the constant-mass-flux controller included, for the
 * members that set it).  For the callers running many small problems in one
 * stream (ensembles, parameter sweeps).  ws_dev must be 256-byte aligned and
 * hip_stream a created stream (graph capture).  Errors: HGKS_E_INVALID for any
 * invalid member config (its index is reported by hgks_last_error), members
 * of different precisions, or work lists beyond 2^30 tiles; HGKS_E_DEVICE.
 * Whole-code FP32 members step on FP32 working copies of their states, which
 * hgks_batch_step fills from the callers' states before its steps and writes
 * back after them, as hgks_step does. */
hgks_status hgks_batch_workspace_size(int32_t n, const hgks_config* cfgs, size_t* bytes);
hgks_status hgks_batch_init(int32_t n, const hgks_config* cfgs, double* const* q_devs, void* ws_dev,
                            size_t ws_bytes, void* hip_stream, hgks_ctx* out);
/* Advance every instance nsteps steps with its own CFL time step (graph
 * replays; asynchronous). */
hgks_status hgks_batch_step(hgks_ctx ctx, int32_t nsteps);
/* Statistics of instance i (synchronises the stream). */
hgks_status hgks_batch_stats(hgks_ctx ctx, int32_t i, hgks_stats_t* out);
/* Launch shapes chosen by the autotuner: info = {instances, flux tile width
 * (faces along x), member-group budget for the reconstruction buffers in MiB
 * (0: all instances in one group), number of groups, flux tiles per stage (3
 * directions), source (1 tuned now, 2 read from the file named by
 * HGKS_TUNE_CACHE), reconstruction tiles per stage (3 directions), cell
 * blocks}. */
hgks_status hgks_batch_info(hgks_ctx ctx, int64_t info[8]);

/* Release the host context (device memory stays the caller's). */
hgks_status hgks_destroy(hgks_ctx ctx);

const char* hgks_status_string(hgks_status s);
/* Detail text of the context's last error; with NULL, of the calling thread's
 * last failure that left no context: hgks_init, hgks_batch_init (whose
 * context is released on failure) or hgks_residual_static ("null context" if
 * none). */
const char* hgks_last_error(hgks_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* HGKS_H */
