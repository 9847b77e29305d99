/*
 * slmpp.h -- C-ABI of the MI355X (gfx950) SL-MPP5/7 Vlasov sweep library.
 *
 * The library advances a phase-space distribution f(x, v) of dimension
 * D = 1, 2 or 3 (a DdDv grid) with the directionally split, conservative
 * semi-Lagrangian scheme of Tanaka, Yoshikawa, Minoshima & Yoshida
 * (arXiv:1702.08521): each one-dimensional sweep builds the CSL flux
 * polynomial (Sec. 2.1.2), applies the monotonicity-preserving constraint
 * (App. A) and the positivity-preserving flux limiter (Sec. 2.1.1), and
 * updates the cell averages in conservative form (Eq. (SL)).  Departure
 * offsets larger than one cell are split into an integer cell shift and a
 * fractional flux.  Around the sweeps sit the velocity moment, the periodic
 * Poisson solve with the 2nd/4th/6th-order Green functions and finite-
 * difference forces (Sec. 2.2, App. C), and the Strang step of
 * Eq. (splitting).
 *
 * Conventions
 *  - All pointers named *_dev are device pointers on the current HIP
 *    device; *_host are host pointers.  The caller owns every buffer it
 *    passes in; the library never frees them.
 *  - f is stored row-major as f[x1]..[xD][v1]..[vD] (vD fastest), in the
 *    storage type of the grid (double or float), prod(nx)*prod(nv) values.
 *  - Spatial fields (rho, phi, one acceleration component) are double
 *    arrays of prod(nx) values, row-major [x1]..[xD].  An acceleration
 *    array "accel" holds D such components back to back (component l at
 *    offset l*prod(nx)).
 *  - Every call that enqueues work does so on the stream given at create,
 *    asynchronously, and returns once the work is enqueued; the calls that
 *    copy to the host (slmpp_get_f, slmpp_diag, slmpp_timing_read,
 *    slmpp_sync) synchronise that stream.
 *  - Arguments are validated on the host before anything is enqueued.  A
 *    failing call returns a non-zero slmpp_status, enqueues nothing and
 *    leaves f unchanged; slmpp_last_error() returns a message.  A fault of
 *    earlier asynchronous work is reported as SLMPP_ERR_DEVICE by the next
 *    synchronising call.
 *  - Calls on one context must not run concurrently from several host
 *    threads.
 */
#ifndef SLMPP_H
#define SLMPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLMPP_ABI_VERSION 3

typedef enum {
  SLMPP_OK = 0,
  SLMPP_ERR_INVALID = 1,   /* bad argument (null pointer, dim out of range, enum value) */
  SLMPP_ERR_SHAPE = 2,     /* inconsistent or oversized grid / array size           */
  SLMPP_ERR_NONFINITE = 3, /* non-finite time step or grid bound                   */
  SLMPP_ERR_WORKSPACE = 4, /* workspace smaller than slmpp_workspace_bytes()       */
  SLMPP_ERR_DEVICE = 5,    /* a HIP call failed                                    */
  SLMPP_ERR_STATE = 6      /* call not valid in the current state                  */
} slmpp_status;

typedef enum { SLMPP_F64 = 0, SLMPP_F32 = 1 } slmpp_dtype;

/* Boundary condition of an axis.  OUTFLOW reads zero outside the domain,
 * so nothing flows in and what crosses the edge leaves the grid. */
typedef enum { SLMPP_BC_PERIODIC = 0, SLMPP_BC_OUTFLOW = 1 } slmpp_bc;

/* Interface flux of a sweep: the CSL polynomial alone, with the MP
 * constraint (SL-MP5/7), or with the MP constraint and the PP limiter
 * (SL-MPP5/7, the paper's production scheme). */
typedef enum { SLMPP_LIM_NONE = 0, SLMPP_LIM_MP = 1, SLMPP_LIM_MPP = 2 } slmpp_limiter;

/* Grid and scheme description.  Entries beyond D are ignored. */
typedef struct {
  int32_t D;             /* spatial dimensions = velocity dimensions, 1..3   */
  int32_t order;         /* 5 (CSL5 / MP5) or 7 (CSL7 / MP7)                  */
  int32_t limiter;       /* slmpp_limiter                                     */
  int32_t poisson_order; /* 2, 4 or 6: Green function and FDA order (App. C)  */
  int64_t nx[3];         /* cells per spatial axis, 1..4096                   */
  int64_t nv[3];         /* cells per velocity axis, 1..4096                  */
  double x_lo[3], x_hi[3]; /* spatial domain, cell centres at lo+(i+1/2)dx    */
  double v_lo[3], v_hi[3]; /* velocity domain                                 */
  double alpha;          /* MP parameter (App. A: alpha = 4), > 0             */
  double kappa;          /* Poisson coupling: lap(phi) = kappa (rho - mean);
                            4 pi G for gravity, -1 for electrons with a
                            neutralising ion background (omega_pe = 1)      */
  int32_t x_bc, v_bc;    /* slmpp_bc of the spatial / velocity axes; the
                            field solve is periodic in space                */
  int32_t storage;       /* slmpp_dtype of f (sweeps compute in this type;
                            moment, Poisson and forces are always double)   */
  int32_t flags;         /* SLMPP_FLAG_* bits (0: none)                     */
} slmpp_grid_desc;

/* flags: time integration of every sweep by the method of lines with the
 * MP(P) interface values and the three-stage TVD Runge-Kutta scheme of
 * Eq. (RK) (RK-MP5/7, RK-MPP5/7, Sec. 2.1.1) instead of the semi-Lagrangian
 * update.  Each sweep then needs |c dt / h| <= 1 (positivity with the PP
 * limiter needs < 1/2): sweeps along x_l are checked on the host
 * (SLMPP_ERR_INVALID); a velocity sweep whose acceleration breaks it writes
 * NaN into the affected pencils (counted by slmpp_diag).  The workspace
 * grows by one copy of f.  Not available for batched ensembles. */
#define SLMPP_FLAG_RK3 1

/* flags: slmpp_step merges, within one call, the closing velocity
 * half-step of a step with the opening half-step of the next (they use the
 * same acceleration) into one velocity sweep with dt: 2D sweeps per step
 * instead of 3D, plus the first and last half-steps of the call.  The
 * state after the call is at the same time level; the splitting stays
 * second order (the result differs from the unmerged one at that order). */
#define SLMPP_FLAG_MERGE_KICKS 2

/* flags: the field solve uses isolated boundaries instead of periodic ones
 * (the doubling-up method of Sec. 2.2: the density is zero-padded to the
 * grid doubled along each axis and convolved with the real-space Green
 * function -kappa / (4 pi r); the cell mean of 1/r at r = 0).  Forces by
 * the FDA of poisson_order on the doubled potential.  D = 3 only; the
 * workspace grows by 40 doubles per spatial cell. */
#define SLMPP_FLAG_ISOLATED 4

/* flags: slmpp_step sweeps every velocity axis of a kick separately.
 * Without it, when D >= 2, the velocity boundaries are outflow, the limiter
 * is SLMPP_LIM_MPP, the time integration semi-Lagrangian and the last two
 * velocity axes have N x N cells with N in {24, 32, 48, 64}, the sweeps
 * along v_{D-1} and v_D of a kick are done in one pass over f (timing class
 * 7), with results equal to the separate sweeps bit for bit. */
#define SLMPP_FLAG_SEPARATE_KICKS 8

typedef struct slmpp_ctx slmpp_ctx;

/* Diagnostics of the current state (Sec. 3: mass, energy, mode amplitude). */
typedef struct {
  double mass;          /* sum f * dx^D dv^D (double, compensated)            */
  double f_min, f_max;  /* extreme cell values of f                            */
  double field_energy;  /* 1/2 sum |a|^2 dx^D of the context's acceleration    */
  double mode_amp;      /* |sum_x a_1(x) exp(-2 pi i x1 / L1)| / prod(nx)     */
  int64_t nonfinite;    /* number of non-finite values of f                    */
} slmpp_diag_out;

/* Per-kernel-class timing gathered with HIP events on the context stream. */
#define SLMPP_TIMING_CLASSES 8 /* 0: sweeps along a strided axis, tiles of
                                     128 or 256 pencils,
                                  1: sweeps along the contiguous axis,
                                  2: velocity moment, 3: Poisson + force,
                                  4: sweeps along a strided axis, other tiles,
                                  5: per-pencil shift / weight tables,
                                  6: x_1 sweeps of slmpp_step that also sum
                                     the velocity moment,
                                  7: the v_{D-1} and v_D sweeps of a kick in
                                     one pass (two cell updates per cell) */
typedef struct {
  int64_t launches[SLMPP_TIMING_CLASSES];
  double total_ms[SLMPP_TIMING_CLASSES];  /* summed kernel durations       */
  double bytes[SLMPP_TIMING_CLASSES];     /* algorithmic HBM bytes summed  */
  double cells[SLMPP_TIMING_CLASSES];     /* cell updates (sweeps) summed  */
} slmpp_timing;

/* ABI version compiled into the library (SLMPP_ABI_VERSION). */
int32_t slmpp_abi_version(void);

/* Device bytes of the workspace a context over `desc` needs (rho, phi,
 * forces, Green table, Fourier buffers, reduction scratch, init staging).
 * Returns 0 when desc is invalid. */
size_t slmpp_workspace_bytes(const slmpp_grid_desc* desc);

/* Check desc without touching the device.  Returns SLMPP_OK or the code
 * create would return; msg (may be NULL) receives the reason. */
slmpp_status slmpp_validate(const slmpp_grid_desc* desc, char* msg, size_t msg_len);

/* Create a context.  f_dev: caller-owned device array of the grid's cells
 * in the storage type, 16-byte aligned; it must stay allocated and unmoved
 * until destroy.
 * work_dev/work_bytes: caller-owned device workspace of at least
 * slmpp_workspace_bytes(desc) bytes, 256-byte aligned.  hip_stream: the
 * hipStream_t all work is enqueued on (NULL = the null stream).  On
 * success *out receives the context; f is not touched. */
slmpp_status slmpp_create(const slmpp_grid_desc* desc, void* f_dev, void* work_dev,
                          size_t work_bytes, void* hip_stream, slmpp_ctx** out);

/* Release the context's own host state (never the caller's buffers). */
slmpp_status slmpp_destroy(slmpp_ctx* ctx);

/* Message of the last failing call on ctx ("" if none); with ctx == NULL,
 * the message of the last failing slmpp_create/validate in this thread. */
const char* slmpp_last_error(const slmpp_ctx* ctx);

/* f <- f_host (n = number of cells, double values, converted to the
 * storage type).  Blocking copy. */
slmpp_status slmpp_init_f_host(slmpp_ctx* ctx, const double* f_host, int64_t n);

/* f(x, v) <- s(x) * g1(v1) * g2(v2) * g3(v3), the product taken left to
 * right in double and rounded once to the storage type.  s_host has
 * prod(nx) values, g_l has nv_l values (NULL for l >= D).  The factors are
 * staged through the workspace. */
slmpp_status slmpp_init_f_separable(slmpp_ctx* ctx, const double* s_host, const double* g1,
                                    const double* g2, const double* g3);

/* One SL step of every pencil along x_dim (dim = 0..D-1) with speed
 * v_dim = the velocity cell centre of the pencil and time step dt
 * (Eq. (adv_pos)).  In place.  dt may be negative (time reversal). */
slmpp_status slmpp_advect_x(slmpp_ctx* ctx, int32_t dim, double dt);

/* One SL step of every pencil along v_dim with speed accel_dev[ix] (the
 * acceleration component at the pencil's spatial cell, prod(nx) doubles on
 * the device), Eq. (adv_vel).  In place. */
slmpp_status slmpp_advect_v(slmpp_ctx* ctx, int32_t dim, double dt, const double* accel_dev);

/* slmpp_advect_v without a context and without any workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  desc describes the grid
 * of f_dev (caller-owned, 16-byte aligned, the grid's cells in its storage
 * type); accel_dev (prod(nx) doubles) and dt as for slmpp_advect_v; the
 * work is enqueued on hip_stream (NULL = the null stream) and the result
 * equals slmpp_advect_v's bit for bit.  The pencil table lives in a 16 MiB
 * device array of the library that each GPU holds from its first call
 * until the process ends: grids whose table (one 48-byte FP32 or 80-byte
 * FP64 entry per spatial cell) exceeds it return SLMPP_ERR_SHAPE.  All
 * calls on one GPU share that array, so calls that overlap on one GPU (on
 * different streams, or from several host threads) race.  Not with
 * SLMPP_FLAG_RK3 (SLMPP_ERR_INVALID).  Errors: slmpp_last_error(NULL). */
slmpp_status slmpp_advect_v_noalloc(const slmpp_grid_desc* desc, void* f_dev, int32_t dim,
                                    double dt, const double* accel_dev, void* hip_stream);

/* One velocity kick: SL steps along v_1, .., v_D in that order, each by dt
 * with the context's acceleration (computed from f first when f changed
 * since the last field solve), as in the half-kicks of slmpp_step: the last
 * two axes in one pass when the two-axis kernel takes the grid (see
 * SLMPP_FLAG_SEPARATE_KICKS).  Leaves the field stale.  In place. */
slmpp_status slmpp_kick(slmpp_ctx* ctx, double dt);

/* rho_dev[ix] <- dv^D * sum_v f(ix, v) (compensated double accumulation). */
slmpp_status slmpp_density_moment(slmpp_ctx* ctx, double* rho_dev);

/* Velocity moments of every spatial cell (Sec. 2.3: density, mean
 * velocities, velocity dispersions), double, on the device:
 *   rho_dev[ix]          = dv^D sum_v f(ix, v)            (prod(nx) values)
 *   mean_dev[l*nxs + ix] = sum_v f v_l / sum_v f          (D*prod(nx))
 *   disp_dev[l*nxs + ix] = sum_v f (v_l - mean_l)^2 / sum_v f (D*prod(nx))
 * with v_l the velocity cell centres and nxs = prod(nx); cells with zero
 * density get zero mean and dispersion.  Compensated accumulation. */
slmpp_status slmpp_velocity_moments(slmpp_ctx* ctx, double* rho_dev, double* mean_dev,
                                    double* disp_dev);

/* Velocity distribution F(v) = dx^D sum_x f(x, v) (Sec. 3.3): F_dev gets
 * prod(nv) doubles on the device, in the layout of one velocity block. */
slmpp_status slmpp_velocity_distribution(slmpp_ctx* ctx, double* F_dev);

/* Periodic Poisson solve lap(phi) = kappa (rho - mean rho) by discrete
 * Fourier transform with the Green function of order poisson_order
 * (Sec. 2.2), then accel_l = -d(phi)/dx_l by the FDA of the same order
 * (App. C).  phi_dev may be NULL.  rho_dev and accel_dev (D*prod(nx)) are
 * device arrays that must not overlap the workspace. */
slmpp_status slmpp_poisson_solve(slmpp_ctx* ctx, const double* rho_dev, double* phi_dev,
                                 double* accel_dev);

/* Recompute the context's own acceleration from the current f
 * (density moment + Poisson solve). */
slmpp_status slmpp_field(slmpp_ctx* ctx);

/* Device pointers of the context's rho, phi and accel arrays (read-only
 * for the caller; valid until destroy).  Any output pointer may be NULL. */
slmpp_status slmpp_field_ptrs(const slmpp_ctx* ctx, const double** rho_dev,
                              const double** phi_dev, const double** accel_dev);

/* Copy the context's rho (prod(nx)) and acceleration (D*prod(nx)) to the
 * host as of the last field computation; either pointer may be NULL.
 * Synchronises. */
slmpp_status slmpp_get_field(slmpp_ctx* ctx, double* rho_host, double* accel_host);

/* One time step of Eq. (splitting): v1..vD with dt/2 using the context's
 * acceleration, xD..x1 with dt, density moment + Poisson, v1..vD with
 * dt/2 using the new acceleration.  If f was changed by any other call
 * since the acceleration was last computed, the acceleration is first
 * recomputed from f.  nsteps >= 1 steps are enqueued back to back. */
slmpp_status slmpp_step(slmpp_ctx* ctx, double dt, int32_t nsteps);

/* Copy f to the host as doubles (n = number of cells).  Synchronises. */
slmpp_status slmpp_get_f(slmpp_ctx* ctx, double* f_host, int64_t n);

/* Diagnostics of f and of the context's acceleration.  Synchronises. */
slmpp_status slmpp_diag(slmpp_ctx* ctx, slmpp_diag_out* out);

/* Wait for all work enqueued on the context's stream. */
slmpp_status slmpp_sync(slmpp_ctx* ctx);

/* Enable (1) or disable (0) per-launch HIP-event timing of the context's
 * kernels, and clear the accumulated figures. */
slmpp_status slmpp_timing_enable(slmpp_ctx* ctx, int32_t on);

/* Read the accumulated timing (synchronises). */
slmpp_status slmpp_timing_read(slmpp_ctx* ctx, slmpp_timing* out);

/* Plain device copy of `bytes` bytes by a streaming kernel (16-byte
 * vectors; both pointers 16-byte aligned, no overlap) on hip_stream.  A
 * reference of known traffic for hardware counters. */
slmpp_status slmpp_copy_device(void* dst_dev, const void* src_dev, size_t bytes,
                               void* hip_stream);

/* Device memory for f (or any caller buffer) on the current device, for
 * callers that want to choose its placement.  contiguous = 1 asks the
 * driver for physically contiguous memory (hipExtMallocWithFlags with
 * hipDeviceMallocContiguous): the strided sweeps then need fewer address
 * translations (measured 1-2% faster per sweep at 48^3 x 48^3 than the
 * same sweep over an ordinary allocation in the same process);
 * contiguous = 0 is a plain hipMalloc.  The caller owns the memory and
 * releases it with slmpp_free_device once no work on it is pending.
 * Errors (*out is set to NULL first, when out is not NULL, and nothing is
 * allocated): out NULL or bytes 0 (SLMPP_ERR_INVALID); the driver cannot
 * provide the memory (SLMPP_ERR_DEVICE).  The contents are undefined. */
slmpp_status slmpp_alloc_device(size_t bytes, int32_t contiguous, void** out);

/* Release memory from slmpp_alloc_device (NULL is accepted and ignored). */
slmpp_status slmpp_free_device(void* p);

/* ------------------------------------------------------------------------
 * Batched ensembles: many independent runs (each with its own grid, order,
 * dt and initial condition) advanced together.  Every phase of the Strang
 * step (Eq. (splitting)) is one grouped launch over all runs -- pencil
 * tables, then a persistent sweep kernel whose work items are tiles of the
 * runs' pencils -- and the field solve is one batched moment launch plus
 * one Poisson workgroup per run.  slmpp_batch_step replays the whole step
 * as one captured HIP graph.
 *
 * Restrictions: all runs share the storage type; limiter SLMPP_LIM_MPP;
 * at most 2048 spatial cells per run (the Poisson solve of a run works in
 * the LDS of one workgroup); dt fixed per run at creation.
 * ------------------------------------------------------------------------ */
typedef struct slmpp_batch slmpp_batch;

/* Device workspace bytes for an ensemble of nruns descriptions (0 when any
 * description is invalid or the runs cannot form a batch). */
size_t slmpp_batch_workspace_bytes(const slmpp_grid_desc* descs, int32_t nruns);

/* Create an ensemble.  f_dev[r]: caller-owned device array of run r
 * (16-byte aligned, prod(nx)*prod(nv) values of the storage type); dts[r]:
 * the run's time step (finite).  work_dev: caller-owned workspace of at
 * least slmpp_batch_workspace_bytes() bytes, 256-byte aligned. */
slmpp_status slmpp_batch_create(const slmpp_grid_desc* descs, const double* dts, int32_t nruns,
                                void* const* f_dev, void* work_dev, size_t work_bytes,
                                void* hip_stream, slmpp_batch** out);
slmpp_status slmpp_batch_destroy(slmpp_batch* b);
/* Message of the last failing call on b; NULL: last failing create. */
const char* slmpp_batch_last_error(const slmpp_batch* b);

/* f_r(x, v) <- s(x) g1(v1) g2(v2) g3(v3) for run r (as slmpp_init_f_separable). */
slmpp_status slmpp_batch_init_separable(slmpp_batch* b, int32_t run, const double* s_host,
                                        const double* g1, const double* g2, const double* g3);

/* Advance every run by nsteps steps of its own dt: the captured step graph
 * is replayed nsteps times (captured on first use, re-captured after
 * slmpp_batch_autotune).  The acceleration of each run is recomputed from
 * f first when an init call changed f.  When the runs carry
 * SLMPP_FLAG_MERGE_KICKS (all or none of them) the call merges kicks as
 * slmpp_step does: an opening half-kick, nsteps - 1 step bodies ending in a
 * full kick and a last one ending in a half-kick (three graphs). */
slmpp_status slmpp_batch_step(slmpp_batch* b, int32_t nsteps);
/* The same launches enqueued directly on the stream, without the graph. */
slmpp_status slmpp_batch_step_eager(slmpp_batch* b, int32_t nsteps);

/* Copy run r's f to the host as doubles (n cells).  Synchronises. */
slmpp_status slmpp_batch_get_f(slmpp_batch* b, int32_t run, double* f_host, int64_t n);

/* Choose the tile width of every distinct pencil shape of the ensemble by
 * timing the candidates (128, 64, 32, 16, 8 pencils per 256-thread tile) on a
 * scratch copy of a run's data.  cache_path (may be NULL) is a text file
 * of "dtype order n inner W" lines: shapes found there are not re-timed,
 * and new choices are appended.  Synchronises. */
slmpp_status slmpp_batch_autotune(slmpp_batch* b, const char* cache_path);

/* Sweeps of runs with one geometry (the same dims, order, boundaries,
 * alpha and largest fast shift) that the persistent single-run kernel
 * takes are advanced by one launch of it per phase when their cells add up
 * to at least min_cells (default 4194304); so are the v_{D-1} and v_D
 * sweeps of the kicks of runs with one velocity-plane geometry that the
 * two-axis pass of slmpp_step takes (see SLMPP_FLAG_SEPARATE_KICKS), as
 * one pass in the v_D phase.  A grouped x_1 phase whose tiles lie within
 * velocity blocks also leaves the tile row sums of the velocity moment
 * (summed per run afterwards instead of a pass over f).  The other sweeps
 * stay in the grouped tile launch.  min_cells < 0: never.  Every sweep
 * gives the same results in all forms, bit for bit; the fused moment sums
 * in another order (equal to rounding).  Rebuilds the launch lists (the
 * step graph is captured again on the next slmpp_batch_step).
 * Synchronises. */
slmpp_status slmpp_batch_set_fast_min_cells(slmpp_batch* b, int64_t min_cells);

/* Algorithmic HBM bytes of one step of the launch lists as built (with
 * merged kicks: of one step body): every pass over a run's f reads and
 * writes it once (a two-axis kick pass counts once for its two sweeps) and
 * the velocity moment reads it once.  For roofline figures; 0 for a NULL
 * batch. */
double slmpp_batch_step_bytes(const slmpp_batch* b);

/* Tile width chosen for run r's sweep along array axis a (0..2D-1): the
 * pencils per tile of the launch that advances it (128, 64, 48, 32, 16 or
 * 8; for the two velocity axes of a two-axis pass, the plane side 24, 32,
 * 48 or 64); 0 when the run has no such axis. */
int32_t slmpp_batch_tile_width(const slmpp_batch* b, int32_t run, int32_t axis);

#ifdef __cplusplus
}
#endif

#endif /* SLMPP_H */
