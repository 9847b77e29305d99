// Internal declarations shared by the HIP translation units of libslmpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "slmpp.h"

namespace slmpp {

// Validation of a grid description shared by single runs and ensembles.
slmpp_status check_grid_desc(const slmpp_grid_desc* d, std::string& msg);

// Speed of a pencil: from the velocity cell centre of the pencil (sweeps
// along x_l) or from an acceleration array indexed by the spatial cell
// (sweeps along v_l).
enum SpeedMode : int32_t { SPEED_FROM_VELOCITY = 0, SPEED_FROM_ACCEL = 1 };

// One sweep over an array viewed as [outer][n][inner]: pencil p = o*inner + j
// holds the elements o*n*inner + i*inner + j, i = 0..n-1.
struct SweepArgs {
  void* f;              // float* or double*
  const double* accel;  // SPEED_FROM_ACCEL: speed of the pencil = accel[(p/inner)/xdiv]
  int64_t npen;         // outer * inner
  int64_t inner;        // stride of the swept axis in elements
  int64_t vdiv;         // SPEED_FROM_VELOCITY: jv = ((p % inner) / vdiv) % nvl
  int64_t xdiv;
  double dt, h;         // time step and mesh spacing of the swept axis
  double vlo, dv;       // velocity axis of SPEED_FROM_VELOCITY
  double alpha;         // MP parameter
  int32_t n;            // pencil length
  int32_t nvl;
  int32_t bc;           // SLMPP_BC_*
  int32_t cmode;        // SpeedMode
  int32_t nfast;        // integer shifts |N| <= nfast read the LDS tile directly
  int32_t rk;           // 1: a TVD-RK stage (interface values at zero Courant
                        //    number, update with nu = c dt / h, no shift)
  double* mom;          // non-null: per-tile sums of the result over each tile row
                        // (strided tiles within one velocity block), mom[tile * n + i]
  // several runs of one geometry in one fast launch (batched ensembles):
  // tile t belongs to run t / tpr, whose f and pencil table are fmulti[r]
  // and tmulti[r] (null: the single run f, table)
  void* const* fmulti;
  const void* const* tmulti;
  int64_t tpr;
  // stages of the TVD-RK time integration (single runs, sweep_fast_kernel
  // and the tile kernels): the results go to fout (null: f, in place),
  // and with fblend non-null each result r becomes cb * fblend + cf * r at
  // the same element
  void* fout;
  const void* fblend;
  double cb, cf;
};

// Tiling of one sweep launch: W pencils per tile, S segments per pencil,
// W*S threads per workgroup, G ghost rows above and below the tile in LDS.
struct SweepPlan {
  int32_t W, S, R, threads, G, pitch;  // R: cells per thread (0: runtime length)
  int32_t fast;                        // use the persistent prefetching kernel
  size_t lds_bytes;
  int64_t tiles;
};

// Plans a sweep launch for the given sizes (dtype: SLMPP_F64/F32); moment:
// the sweep also leaves tile row sums (SweepArgs::mom) when its plan allows.
SweepPlan plan_sweep(int dtype, int order, int limiter, int32_t n, int64_t npen, int64_t inner,
                     int32_t nfast, int W_override = 0, int S_override = 0, bool moment = false);

// Enqueue the pencil table (table_count entries, one per distinct speed;
// `table` is device scratch of pencil_table_bytes()), then the sweep.
hipError_t launch_pencil_table(int dtype, int order, const SweepArgs& a, void* table,
                               int64_t table_count, hipStream_t s);
hipError_t launch_sweep(int dtype, int order, int limiter, const SweepArgs& a,
                        const SweepPlan& p, const void* table, hipStream_t s);
size_t pencil_table_bytes(int dtype, int64_t count);

// The last two velocity axes of one kick in one pass over f (outflow
// velocity boundaries, SL-MPP, square planes of N = 24, 32, 48 or 64
// cells): plane p = (x, v_1..v_{D-2}) is the contiguous block
// f[p * N^2 .. (p + 1) * N^2); its pencils along v_{D-1} take table entry
// tabA[p / vouter] and those along v_D tabB[p / vouter].  Several runs of
// one geometry in one launch: SweepArgs::fmulti / tmulti / tpr (tiles per
// run) with tmulti holding the v_{D-1} tables of the runs, then their v_D
// tables; planes and tiles as for one run, times the number of runs for
// tiles.
// n / d for 32-bit n by an invariant 32-bit divisor d >= 1 (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994):
// t = mulhi(m, n), n / d = (t + ((n - t) >> s1)) >> s2 with
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0).  m == 0 marks "not set up".
struct FastDiv32 {
  uint32_t m, s1, s2, pad;
  static FastDiv32 of(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;
    FastDiv32 f{};
    f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
  }
  __host__ __device__ uint32_t div(uint32_t n) const {
    const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
    return (t + ((n - t) >> s1)) >> s2;
  }
};

struct PlanePlan {
  int32_t N, PB;       // plane side, planes per tile
  int32_t G, pitch;    // ring of zero cells around each plane in LDS, LDS row
                       // pitch (fixed by order and N; shifts beyond the ring
                       // minus the stencil take bounds-checked reads)
  int32_t plane_lds;   // LDS elements from one plane to the next
  int32_t uni;         // the planes of a tile share one spatial cell (vouter % PB == 0)
  int64_t planes, vouter, tiles;
  FastDiv32 vdiv;      // plane -> spatial cell (plane / vouter) while planes < 2^32
  size_t lds_bytes;    // 0: the shape is not supported
};
PlanePlan plan_kick_plane(int dtype, int order, int32_t na, int32_t nb, int64_t planes,
                          int64_t vouter);
hipError_t launch_kick_plane(int dtype, int order, const SweepArgs& a, const PlanePlan& p,
                             const void* tabA, const void* tabB, hipStream_t s);

// Integer-shift bound of a sweep along x_l: max |N| over the velocity
// centres of axis l, with the same split as the kernels.
int32_t max_shift_velocity(double vlo, double dv, int32_t nvl, double dt, double h, int32_t n,
                           int32_t bc);

// ---- batched ensembles (many independent runs per launch) ----
// One sweep of one run inside a grouped launch.
struct BatchSweep {
  SweepArgs a;
  SweepPlan p;
  void* table;    // the run's pencil-table scratch
  int32_t order;  // 5 or 7
  int32_t count;  // table entries
};
// One work item of a grouped sweep launch: tile `tile` of sweep `sweep`.
struct BatchItem {
  int32_t sweep;
  int32_t pad;
  int64_t tile;
};
// Field data of one run.
struct BatchRun {
  const void* f;
  double* rho;
  double* phi;
  double* accel;
  int64_t nxs, nvs;
  int64_t nx[3];
  double h[3];
  double dvol;
  double kappa;
  int32_t D;
  int32_t poisson_order;
};
// rho of one run from the tile row sums of its x_1 sweep (fused moment):
// rho[i * ncol + c] = dvol * sum_{q < nsub} part[(c * nsub + q) * n + i]
struct BatchReduce {
  const double* part;
  double* rho;
  int64_t ncol, nsub;
  int32_t n, pad;
  double dvol;
};
hipError_t launch_batch_reduce(const BatchReduce* list, int nlist, int64_t max_cells,
                               hipStream_t s);
hipError_t launch_batch_tables(int dtype, const BatchSweep* sweeps, int nsweeps, int max_count,
                               hipStream_t s);
hipError_t launch_batch_sweeps(int dtype, const BatchSweep* sweeps, const BatchItem* items,
                               int nitems, size_t lds_bytes, int grid, hipStream_t s);
int batch_sweep_blocks_per_cu(int dtype, size_t lds_bytes);
SweepPlan plan_batch_sweep(int dtype, int order, int32_t n, int64_t npen, int64_t inner,
                           int32_t nfast, int W);
hipError_t launch_generic_sweep(int dtype, int order, const SweepArgs& a, const SweepPlan& p,
                                const void* table, hipStream_t s);
hipError_t launch_batch_moment(int dtype, const BatchRun* runs, const int2* items, int nitems,
                               hipStream_t s);
hipError_t launch_batch_poisson(const BatchRun* runs, int nruns, int max_nxs, hipStream_t s);
// Kernel attributes for the LDS sizes of a batch (outside any graph capture).
hipError_t prepare_batch_kernels(int dtype, size_t sweep_lds, int max_nxs);
constexpr int kBatchMaxSpace = 2048;  // spatial cells per run (one-workgroup Poisson)
// LDS of one batch tile: preferred budget (at least five 256-thread
// workgroups per CU) and hard limit
constexpr size_t kBatchTileLds = 32 * 1024;
constexpr size_t kBatchTileLdsMax = 96 * 1024;

// ---- field kernels (field.hip) ----
hipError_t launch_moment(int dtype, const void* f, int64_t nxs, int64_t nvs, double dvol,
                         double* rho, hipStream_t s);
// rho[i * ncol + c] = dvol * sum_{q < nsub} part[(c * nsub + q) * n + i]: the
// velocity moment from the row sums of a fused x_1 sweep (ncol spatial
// columns of x_2..x_D, nsub tiles per velocity block).
hipError_t launch_moment_reduce(const double* part, int n, int64_t ncol, int64_t nsub, double dvol,
                                double* rho, hipStream_t s);
hipError_t launch_poisson(const double* rho, double* phi, double* accel, double2* bufA,
                          double2* bufB, const double2* twiddles, const int64_t* tw_off,
                          const double* green, int D, const int64_t* nx, const double* h,
                          int order, hipStream_t s);
// isolated boundaries (D = 3): Fourier transform of the real-space Green
// function held in a (as complex, doubled grid of sizes m), real part to
// ghat; the solve itself with a, b as scratch of the doubled size
hipError_t launch_iso_green(double2* a, double2* b, const double2* tw, const int64_t* tw_off,
                            const int64_t* m, double* ghat, hipStream_t s);
hipError_t launch_poisson_isolated(const double* rho, double* phi, double* accel, double2* a,
                                   double2* b, const double2* tw, const int64_t* tw_off,
                                   const double* ghat, const int64_t* nx, const double* h,
                                   int order, hipStream_t s);
hipError_t launch_init_separable(int dtype, void* f, const double* s, const double* g1,
                                 const double* g2, const double* g3, int D, const int64_t* nv,
                                 int64_t nxs, int64_t nvs, hipStream_t st);
hipError_t launch_from_double(int dtype, void* f, const double* src, int64_t n, hipStream_t s);
hipError_t launch_to_double(int dtype, const void* f, double* dst, int64_t n, hipStream_t s);
hipError_t launch_diag_f(int dtype, const void* f, int64_t n, double* partials, int nblocks,
                         hipStream_t s);
hipError_t launch_diag_field(const double* accel, int D, int64_t nxs, int64_t nx1, int64_t inner1,
                             double* out, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// velocity moments per spatial cell and the velocity distribution (double)
hipError_t launch_velocity_moments(int dtype, const void* f, int D, const int64_t* nv,
                                   const double* vlo, const double* dv, int64_t nxs,
                                   double* rho, double* mean, double* disp, hipStream_t s);
hipError_t launch_velocity_distribution(int dtype, const void* f, int64_t nxs, int64_t nvs,
                                        double xvol, double* F, hipStream_t s);
constexpr int kDiagBlocks = 1024;

}  // namespace slmpp
