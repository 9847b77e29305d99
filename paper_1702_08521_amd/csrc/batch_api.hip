// Host runtime of batched ensembles (slmpp_batch_* in include/slmpp.h):
// per-run workspace layout, grouped launch lists for every phase of the
// Strang step, the captured step graph, and the tile-width autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "slmpp_internal.hpp"

using namespace slmpp;

namespace {

thread_local std::string g_batch_error;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct RunGeom {
  int D;
  int64_t dims[6];
  int64_t nxs, nvs, ncell;
  double hx[3], hv[3];
};

RunGeom geom_of(const slmpp_grid_desc& d) {
  RunGeom g{};
  g.D = d.D;
  g.nxs = 1;
  g.nvs = 1;
  for (int l = 0; l < d.D; ++l) {
    g.dims[l] = d.nx[l];
    g.dims[d.D + l] = d.nv[l];
    g.nxs *= d.nx[l];
    g.nvs *= d.nv[l];
    g.hx[l] = (d.x_hi[l] - d.x_lo[l]) / (double)d.nx[l];
    g.hv[l] = (d.v_hi[l] - d.v_lo[l]) / (double)d.nv[l];
  }
  g.ncell = g.nxs * g.nvs;
  return g;
}

// One phase of the step: a sweep along v_l (half step) or x_l (full step).
struct SlotDef {
  bool vel;
  int l;
  double frac;  // fraction of dt
};

// Phases of a step, in groups of Dmax: opening half-kick v_1..v_Dmax,
// x_Dmax..x_1 (full step), closing half-kick; with merged kicks also a
// full kick (a closing and the next opening half-kick in one).
std::vector<SlotDef> slot_defs(int Dmax, bool merged) {
  std::vector<SlotDef> s;
  for (int l = 0; l < Dmax; ++l) s.push_back({true, l, 0.5});
  for (int l = Dmax - 1; l >= 0; --l) s.push_back({false, l, 1.0});
  for (int l = 0; l < Dmax; ++l) s.push_back({true, l, 0.5});
  if (merged)
    for (int l = 0; l < Dmax; ++l) s.push_back({true, l, 1.0});
  return s;
}

const int kCandidates[] = {128, 64, 32, 16, 8};
constexpr int kMinW = 8;

struct Layout {
  std::vector<size_t> rho, phi, acc, tab, tab2;
  // the pencil tables of the step, computed outside the sweep phases: per
  // run and axis l, xt[r * 3 + l] for the x_l sweeps (fixed: dt does not
  // change) and vt[(r * 3 + l) * 2 + k] for the v_l sweeps with dt / 2
  // (k = 0) and, with merged kicks, dt (k = 1) (after every field solve)
  std::vector<size_t> xt, vt;
  size_t tsweeps;  // BatchSweep lists of those table computations
  size_t runs, sweeps, items, mitems, mitems2, mom, reduce, ptrs, scratch, stage, total;
  int64_t max_sweeps, max_items, nmitems, stage_doubles, mom_doubles;
};

Layout layout_of(const std::vector<slmpp_grid_desc>& d) {
  const bool merged = !d.empty() && (d[0].flags & SLMPP_FLAG_MERGE_KICKS) != 0;
  const int kicks = merged ? 3 : 2;  // velocity phases per axis
  Layout L{};
  const int n = (int)d.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  int Dmax = 1;
  int64_t max_cells = 1, stage = 1;
  L.max_items = 0;
  L.nmitems = 0;
  L.mom_doubles = 0;
  for (int r = 0; r < n; ++r) {
    const RunGeom g = geom_of(d[r]);
    Dmax = std::max(Dmax, g.D);
    L.rho.push_back(take(8 * g.nxs));
    L.phi.push_back(take(8 * g.nxs));
    L.acc.push_back(take(8 * g.nxs * g.D));
    int64_t maxnv = 1, sumnv = 0;
    for (int l = 0; l < g.D; ++l) {
      maxnv = std::max<int64_t>(maxnv, d[r].nv[l]);
      sumnv += d[r].nv[l];
    }
    L.tab.push_back(take(pencil_table_bytes(SLMPP_F64, std::max(maxnv, g.nxs))));
    // v_{D-1} table of a two-axis kick pass
    L.tab2.push_back(take(g.D >= 2 ? pencil_table_bytes(SLMPP_F64, g.nxs) : 0));
    for (int l = 0; l < 3; ++l) {
      L.xt.push_back(l < g.D ? take(pencil_table_bytes(SLMPP_F64, d[r].nv[l])) : 0);
      for (int k = 0; k < 2; ++k)
        L.vt.push_back(l < g.D && (k == 0 || merged) ? take(pencil_table_bytes(SLMPP_F64, g.nxs)) : 0);
    }
    // work items: every sweep of a step at the smallest tile width
    for (int a = 0; a < 2 * g.D; ++a) {
      const int64_t npen = g.ncell / g.dims[a];
      L.max_items += (a >= g.D ? kicks : 1) * ((npen + kMinW - 1) / kMinW);
    }
    L.nmitems += g.nxs;
    // row sums of a fused x_1 sweep: tiles of >= 64 pencils, or chunks of
    // 8 velocity cells for 1D1V runs in the tile launch
    L.mom_doubles += g.ncell / (g.D == 1 ? 8 : 64) + 1;
    max_cells = std::max(max_cells, g.ncell);
    stage = std::max(stage, g.nxs + sumnv);
  }
  L.max_sweeps = (int64_t)n * (1 + kicks) * Dmax + 2 * (int64_t)n;
  L.tsweeps = take(sizeof(BatchSweep) * 9 * (size_t)n);
  L.runs = take(sizeof(BatchRun) * n);
  L.sweeps = take(sizeof(BatchSweep) * L.max_sweeps);
  L.items = take(sizeof(BatchItem) * std::max<int64_t>(L.max_items, 1));
  L.mitems = take(sizeof(int2) * std::max<int64_t>(L.nmitems, 1));
  L.mitems2 = take(sizeof(int2) * std::max<int64_t>(L.nmitems, 1));  // runs without a fused moment
  L.mom = take(sizeof(double) * L.mom_doubles);
  L.reduce = take(sizeof(BatchReduce) * n);
  // f and table pointers of persistent launches over several runs
  L.ptrs = take(sizeof(void*) * 4 * L.max_sweeps);
  L.scratch = take(8 * max_cells);
  L.stage_doubles = std::max<int64_t>(stage, std::min<int64_t>(max_cells, (int64_t)1 << 22));
  L.stage = take(8 * L.stage_doubles);
  L.total = off;
  return L;
}

slmpp_status check_batch(const slmpp_grid_desc* descs, int32_t nruns, std::string& msg) {
  if (!descs || nruns < 1) {
    msg = "descs must be non-NULL and nruns >= 1";
    return SLMPP_ERR_INVALID;
  }
  for (int r = 0; r < nruns; ++r) {
    slmpp_status st = check_grid_desc(&descs[r], msg);
    if (st != SLMPP_OK) {
      msg = "run " + std::to_string(r) + ": " + msg;
      return st;
    }
    if (descs[r].storage != descs[0].storage) {
      msg = "all runs of a batch must share the storage type";
      return SLMPP_ERR_INVALID;
    }
    if (descs[r].limiter != SLMPP_LIM_MPP ||
        (descs[r].flags != 0 && descs[r].flags != SLMPP_FLAG_MERGE_KICKS)) {
      msg = "batched runs use the SL-MPP scheme (SLMPP_LIM_MPP; flags 0 or SLMPP_FLAG_MERGE_KICKS)";
      return SLMPP_ERR_INVALID;
    }
    if (descs[r].flags != descs[0].flags) {
      msg = "all runs of a batch must share the flags";
      return SLMPP_ERR_INVALID;
    }
    if (geom_of(descs[r]).nxs > kBatchMaxSpace) {
      msg = "run " + std::to_string(r) + " has more than 2048 spatial cells";
      return SLMPP_ERR_SHAPE;
    }
  }
  return SLMPP_OK;
}

std::string shape_key(int dtype, int order, int64_t n, int64_t inner) {
  std::ostringstream o;
  o << (dtype == SLMPP_F64 ? "f64" : "f32") << ' ' << order << ' ' << n << ' ' << inner;
  return o.str();
}

// Everything the persistent kernel takes from the sweep arguments besides
// f and the pencil table: sweeps with equal keys can share one launch.
std::string fast_key(int order, const SweepArgs& a) {
  std::ostringstream o;
  o << order << ' ' << a.n << ' ' << a.npen << ' ' << a.inner << ' ' << a.nfast << ' ' << a.bc << ' '
    << a.cmode << ' ' << a.xdiv << ' ' << a.vdiv << ' ' << a.nvl << ' ' << std::hexfloat << a.alpha;
  return o.str();
}

// Default of slmpp_batch_set_fast_min_cells: 16 MiB of FP32 data
constexpr int64_t kFastMinCells = (int64_t)1 << 22;

}  // namespace

struct slmpp_batch {
  int nruns = 0, dtype = SLMPP_F32, Dmax = 1;
  bool merged = false;  // SLMPP_FLAG_MERGE_KICKS (every run)
  hipStream_t stream = nullptr;
  std::vector<slmpp_grid_desc> d;
  std::vector<RunGeom> g;
  std::vector<double> dt;
  std::vector<void*> f;
  char* work = nullptr;
  size_t work_bytes = 0;
  Layout lay{};
  std::vector<SlotDef> slots;
  struct SlotLaunch {
    int first_sweep, nsweeps, first_item, nitems, max_count, grid, first_group, ngroups;
    size_t lds;
    int first_pgroup, npgroups;
  };
  std::vector<SlotLaunch> launches;
  // runs of one geometry advanced by one launch of the persistent kernel
  struct FastGroup {
    int order;
    SweepArgs a;  // fmulti / tmulti / tpr set
    SweepPlan p;  // tiles over all runs of the group
  };
  std::vector<FastGroup> groups;
  // velocity moment fused into the x_1 sweep of fast groups: the runs'
  // row-sum reductions, and the moment items of the other runs
  std::vector<BatchReduce> reduce;
  std::vector<int2> mitems2;
  int64_t max_reduce_cells = 0;
  // runs of one plane geometry whose v_{D-1} and v_D sweeps of a kick run
  // as one kick_plane_kernel launch (in the v_D phase)
  struct PlaneGroup {
    int order;
    SweepArgs a;  // alpha, fmulti / tmulti / tpr
    PlanePlan p;  // tiles over all runs of the group
  };
  std::vector<PlaneGroup> pgroups;
  double step_bytes = 0.0;  // algorithmic HBM bytes of one step as built
  std::vector<double> slot_bytes;
  std::vector<void*> group_ptrs;
  int64_t fast_min_cells = kFastMinCells;
  std::vector<BatchSweep> sweeps;
  std::vector<BatchItem> items;
  std::vector<BatchRun> runs;
  std::map<std::string, int> width;  // shape key -> tile width
  std::vector<int> run_axis_width;   // run * 6 + axis
  int max_nxs = 1;
  size_t max_lds = 0;
  // captured graphs by kind: 0 a whole step; with merged kicks 1 the
  // opening half-kick, 2 a step body ending in a full kick, 3 the last step
  // body ending in a half-kick
  hipGraph_t graph[4] = {};
  hipGraphExec_t exec[4] = {};
  hipStream_t capture = nullptr;  // private stream the step graph is captured on
  bool field_valid = false;
  std::string err;

  slmpp_status fail(slmpp_status code, const std::string& m) {
    err = m;
    return code;
  }
  slmpp_status hip_fail(hipError_t e, const char* what) {
    return fail(SLMPP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
  template <typename T>
  T* at(size_t off) {
    return reinterpret_cast<T*>(work + off);
  }

  // The pencil table of run r for a sweep of slot kind sd (see Layout::xt, vt).
  void* table_of(int r, const SlotDef& sd) {
    if (!sd.vel) return work + lay.xt[(size_t)r * 3 + sd.l];
    return work + lay.vt[((size_t)r * 3 + sd.l) * 2 + (sd.frac == 1.0 ? 1 : 0)];
  }
  // table computations done outside the phases: the x tables once per
  // build, the v tables after every field solve (BatchSweep lists at
  // lay.tsweeps: nxt x entries, then nvt v entries)
  int nxt = 0, nvt = 0, xt_max = 0, vt_max = 0;

  // Sweep arguments of run r for slot s (nullptr-table entries filled in).
  bool sweep_of(int r, const SlotDef& sd, SweepArgs& a, int64_t& count) const {
    const RunGeom& G = g[r];
    if (sd.l >= G.D) return false;
    const int axis = sd.vel ? G.D + sd.l : sd.l;
    const int nd = 2 * G.D;
    int64_t inner = 1, outer = 1;
    for (int k = axis + 1; k < nd; ++k) inner *= G.dims[k];
    for (int k = 0; k < axis; ++k) outer *= G.dims[k];
    a = SweepArgs{};
    a.f = f[r];
    a.npen = outer * inner;
    a.inner = inner;
    a.n = (int32_t)G.dims[axis];
    a.dt = sd.frac * dt[r];
    a.alpha = d[r].alpha;
    if (!sd.vel) {
      int64_t vdiv = 1;
      for (int k = G.D + sd.l + 1; k < nd; ++k) vdiv *= G.dims[k];
      a.cmode = SPEED_FROM_VELOCITY;
      a.vdiv = vdiv;
      a.nvl = (int32_t)d[r].nv[sd.l];
      a.vlo = d[r].v_lo[sd.l];
      a.dv = G.hv[sd.l];
      a.h = G.hx[sd.l];
      a.bc = d[r].x_bc;
      a.xdiv = 1;
      a.nfast = max_shift_velocity(a.vlo, a.dv, a.nvl, a.dt, a.h, a.n, a.bc);
      count = d[r].nv[sd.l];
    } else {
      int64_t xdiv = 1;
      for (int k = G.D; k < axis; ++k) xdiv *= G.dims[k];
      a.cmode = SPEED_FROM_ACCEL;
      a.accel = reinterpret_cast<const double*>(work + lay.acc[r]) + (int64_t)sd.l * G.nxs;
      a.xdiv = xdiv;
      a.vdiv = 1;
      a.nvl = 1;
      a.h = G.hv[sd.l];
      a.bc = d[r].v_bc;
      a.nfast = 4;
      count = G.nxs;
    }
    return true;
  }

  // Without timings: the widest tile within the LDS budget, register
  // variants first; else the tile of least LDS.
  int default_width(int order, const SweepArgs& a) const {
    for (int pass = 0; pass < 2; ++pass)
      for (int W : kCandidates) {
        SweepPlan p = plan_batch_sweep(dtype, order, a.n, a.npen, a.inner, a.nfast, W);
        if (p.lds_bytes && p.lds_bytes <= kBatchTileLds && (pass == 1 || p.R > 0)) return W;
      }
    int bestW = 0;
    size_t least = 0;
    for (int W : kCandidates) {
      SweepPlan p = plan_batch_sweep(dtype, order, a.n, a.npen, a.inner, a.nfast, W);
      if (p.lds_bytes && (!bestW || p.lds_bytes < least)) {
        bestW = W;
        least = p.lds_bytes;
      }
    }
    return bestW;
  }

  // Build the grouped launch lists from the current tile widths and upload.
  slmpp_status build() {
    sweeps.clear();
    items.clear();
    launches.clear();
    groups.clear();
    pgroups.clear();
    group_ptrs.clear();
    reduce.clear();
    max_reduce_cells = 0;
    std::vector<char> mom_fused((size_t)nruns, 0);
    std::vector<int64_t> rowsums((size_t)nruns, 0);
    double* mom_next = at<double>(lay.mom);
    const double es = dtype == SLMPP_F64 ? 8.0 : 4.0;
    slot_bytes.assign(slots.size(), 0.0);
    run_axis_width.assign((size_t)nruns * 6, 0);
    max_lds = 0;
    void** dptrs = at<void*>(lay.ptrs);
    // two-axis kick passes: runs with one plane geometry (D >= 2, outflow
    // velocity boundaries, square planes the plane kernel takes) whose
    // cells add up to at least fast_min_cells
    std::vector<int> plane_of((size_t)nruns, -1);
    std::vector<std::vector<int>> pruns;
    std::vector<PlanePlan> pplan;
    if (fast_min_cells >= 0) {
      std::map<std::string, int> pk;
      for (int r = 0; r < nruns; ++r) {
        const int D = g[r].D;
        if (D < 2 || d[r].v_bc != SLMPP_BC_OUTFLOW) continue;
        int64_t vouter = 1;
        for (int l = 0; l < D - 2; ++l) vouter *= d[r].nv[l];
        const PlanePlan pp = plan_kick_plane(dtype, d[r].order, (int32_t)d[r].nv[D - 2],
                                             (int32_t)d[r].nv[D - 1], g[r].nxs * vouter, vouter);
        if (!pp.lds_bytes) continue;
        std::ostringstream o;
        o << D << ' ' << d[r].order << ' ' << pp.N << ' ' << pp.planes << ' ' << vouter << ' '
          << std::hexfloat << d[r].alpha;
        auto it = pk.find(o.str());
        if (it == pk.end()) {
          it = pk.emplace(o.str(), (int)pruns.size()).first;
          pruns.emplace_back();
          pplan.push_back(pp);
        }
        pruns[(size_t)it->second].push_back(r);
      }
      for (size_t q = 0; q < pruns.size(); ++q) {
        int64_t cells = 0;
        for (int r : pruns[q]) cells += g[r].ncell;
        if (cells >= fast_min_cells)
          for (int r : pruns[q]) plane_of[r] = (int)q;
      }
    }
    for (size_t si = 0; si < slots.size(); ++si) {
      SlotLaunch L{(int)sweeps.size(), 0, (int)items.size(), 0, 0, 1, (int)groups.size(), 0, 0,
                   (int)pgroups.size(), 0};
      std::vector<int> pg_here;  // plane groups launched in this phase
      // fast groups: sweeps the persistent kernel takes, of runs with one
      // geometry, whose cells add up to at least fast_min_cells
      std::vector<SweepArgs> args((size_t)nruns);
      std::vector<int64_t> counts((size_t)nruns, 0);
      std::vector<char> has((size_t)nruns, 0);
      std::vector<SweepPlan> fplan((size_t)nruns);
      std::vector<char> grouped((size_t)nruns, 0);
      std::map<std::string, std::vector<int>> by_key;
      for (int r = 0; r < nruns; ++r) {
        has[r] = sweep_of(r, slots[si], args[r], counts[r]);
        if (has[r] && plane_of[r] >= 0 && slots[si].vel && slots[si].l >= g[r].D - 2) {
          // v_{D-1}: done with v_D; v_D: the two tables now, the pass below
          has[r] = 0;
          if (slots[si].l == g[r].D - 1) {
            const int q = plane_of[r];
            if (std::find(pg_here.begin(), pg_here.end(), q) == pg_here.end()) pg_here.push_back(q);
            SlotDef sa = slots[si];
            sa.l = g[r].D - 2;
            BatchSweep ta{}, tb{};
            int64_t ca = 0;
            sweep_of(r, sa, ta.a, ca);
            ta.table = table_of(r, sa);
            ta.order = d[r].order;
            ta.count = (int32_t)ca;
            tb.a = args[r];
            tb.table = table_of(r, slots[si]);
            tb.order = d[r].order;
            tb.count = (int32_t)counts[r];
            sweeps.push_back(ta);
            sweeps.push_back(tb);
            L.nsweeps += 2;
            L.max_count = std::max<int>(L.max_count, (int)std::max(ca, counts[r]));
            run_axis_width[(size_t)r * 6 + 2 * g[r].D - 2] = pplan[(size_t)q].N;
            run_axis_width[(size_t)r * 6 + 2 * g[r].D - 1] = pplan[(size_t)q].N;
          }
          continue;
        }
        if (has[r]) slot_bytes[si] += 2.0 * es * (double)g[r].ncell;
        if (!has[r] || fast_min_cells < 0) continue;
        const SweepArgs& a = args[r];
        fplan[r] = plan_sweep(dtype, d[r].order, SLMPP_LIM_MPP, a.n, a.npen, a.inner, a.nfast, 0, 0,
                              !slots[si].vel && slots[si].l == 0);
        if (fplan[r].fast) by_key[fast_key(d[r].order, a)].push_back(r);
      }
      for (const auto& kv : by_key) {
        const std::vector<int>& rs = kv.second;
        int64_t cells = 0;
        for (int r : rs) cells += g[r].ncell;
        if (cells < fast_min_cells) continue;
        const int r0 = rs[0];
        FastGroup fg{};
        fg.order = d[r0].order;
        fg.a = args[r0];
        fg.p = fplan[r0];
        fg.a.tpr = fplan[r0].tiles;
        fg.p.tiles = fplan[r0].tiles * (int64_t)rs.size();
        const size_t off = group_ptrs.size();
        for (int r : rs) group_ptrs.push_back(f[r]);
        for (int r : rs) group_ptrs.push_back(table_of(r, slots[si]));
        fg.a.fmulti = dptrs + off;
        fg.a.tmulti = const_cast<const void* const*>(dptrs + off + rs.size());
        for (int r : rs) grouped[r] = 1;
        // the x_1 phase of runs whose tiles lie within velocity blocks
        // also leaves the row sums of the velocity moment
        const SweepPlan& fp = fplan[r0];
        const bool x1 = !slots[si].vel && slots[si].l == 0;
        if (x1 && fp.W >= 64 && fg.a.inner > 1 && g[r0].nvs % fp.W == 0) {
          fg.a.mom = mom_next;
          for (size_t k = 0; k < rs.size(); ++k) {
            const int r = rs[k];
            BatchReduce br{};
            br.part = mom_next + (int64_t)k * fp.tiles * fg.a.n;
            br.rho = at<double>(lay.rho[r]);
            br.n = fg.a.n;
            br.ncol = g[r].nxs / fg.a.n;
            br.nsub = g[r].nvs / fp.W;
            br.dvol = runs[r].dvol;
            reduce.push_back(br);
            mom_fused[r] = 1;
            rowsums[r] = fp.tiles * fg.a.n;
            max_reduce_cells = std::max(max_reduce_cells, g[r].nxs);
          }
          mom_next += (int64_t)rs.size() * fp.tiles * fg.a.n;
        }
        groups.push_back(fg);
        ++L.ngroups;
      }
      for (int r = 0; r < nruns; ++r) {
        if (!has[r]) continue;
        const SweepArgs& a = args[r];
        const int64_t count = counts[r];
        const int axis = slots[si].vel ? g[r].D + slots[si].l : slots[si].l;
        if (grouped[r]) {
          // the table is still computed with the slot's other sweeps
          run_axis_width[(size_t)r * 6 + axis] = fplan[r].W;
          BatchSweep b{};
          b.a = a;
          b.p = fplan[r];
          b.table = table_of(r, slots[si]);
          b.order = d[r].order;
          b.count = (int32_t)count;
          sweeps.push_back(b);
          L.max_count = std::max<int>(L.max_count, (int)count);
          ++L.nsweeps;
          continue;
        }
        const std::string key = shape_key(dtype, d[r].order, a.n, a.inner);
        // a width from the autotuner or its cache, else (or when it does
        // not fit this shape) the default
        int W = width.count(key) ? width[key] : 0;
        SweepPlan p{};
        if (W) p = plan_batch_sweep(dtype, d[r].order, a.n, a.npen, a.inner, a.nfast, W);
        if (!p.lds_bytes) {
          W = default_width(d[r].order, a);
          if (W) p = plan_batch_sweep(dtype, d[r].order, a.n, a.npen, a.inner, a.nfast, W);
        }
        if (!p.lds_bytes)
          return fail(SLMPP_ERR_SHAPE, "run " + std::to_string(r) + ": pencils of " +
                                           std::to_string(a.n) + " cells do not fit a batch tile");
        run_axis_width[(size_t)r * 6 + axis] = W;
        BatchSweep b{};
        b.a = a;
        b.p = p;
        b.table = table_of(r, slots[si]);
        b.order = d[r].order;
        b.count = (int32_t)count;
        // the x_1 sweep of a 1D1V run leaves the velocity moment's row sums
        // in chunks of 8 velocity cells (the same for every tile width)
        if (!slots[si].vel && slots[si].l == 0 && g[r].D == 1 && p.W % 8 == 0 &&
            g[r].nvs % 8 == 0) {
          b.a.mom = mom_next;
          BatchReduce br{};
          br.part = mom_next;
          br.rho = at<double>(lay.rho[r]);
          br.n = a.n;
          br.ncol = 1;
          br.nsub = g[r].nvs / 8;
          br.dvol = runs[r].dvol;
          reduce.push_back(br);
          mom_fused[r] = 1;
          rowsums[r] = g[r].ncell / 8;
          max_reduce_cells = std::max(max_reduce_cells, g[r].nxs);
          mom_next += g[r].ncell / 8;
        }
        const int sidx = (int)sweeps.size();
        sweeps.push_back(b);
        for (int64_t t = 0; t < p.tiles; ++t) items.push_back(BatchItem{sidx, 0, t});
        L.max_count = std::max<int>(L.max_count, (int)count);
        L.lds = std::max(L.lds, p.lds_bytes);
        ++L.nsweeps;
      }
      for (int q : pg_here) {
        const std::vector<int>& rs = pruns[(size_t)q];
        const int r0 = rs[0];
        PlaneGroup pg{};
        pg.order = d[r0].order;
        pg.a.alpha = d[r0].alpha;
        pg.a.nfast = 4;
        pg.p = pplan[(size_t)q];
        pg.a.tpr = pg.p.tiles;
        pg.p.tiles *= (int64_t)rs.size();
        const size_t off = group_ptrs.size();
        for (int r : rs) group_ptrs.push_back(f[r]);
        for (int r : rs) slot_bytes[si] += 2.0 * es * (double)g[r].ncell;
        for (int r : rs) group_ptrs.push_back(table_of(r, SlotDef{true, g[r].D - 2, slots[si].frac}));
        for (int r : rs) group_ptrs.push_back(table_of(r, slots[si]));
        pg.a.fmulti = dptrs + off;
        pg.a.tmulti = const_cast<const void* const*>(dptrs + off + rs.size());
        pgroups.push_back(pg);
        ++L.npgroups;
      }
      L.nitems = (int)items.size() - L.first_item;
      max_lds = std::max(max_lds, L.lds);
      launches.push_back(L);
    }
    // one step: the phases of a Strang step (with merged kicks a step body:
    // x phases and a full kick), and the velocity moment (a read of f, or
    // the row sums written and read back when fused into the x_1 phase)
    step_bytes = 0.0;
    for (int r = 0; r < nruns; ++r)
      step_bytes += mom_fused[r] ? 16.0 * (double)rowsums[r] : es * (double)g[r].ncell;
    for (size_t si = 0; si < slots.size(); ++si) {
      const bool in_step = merged ? (int)si >= Dmax && ((int)si < 2 * Dmax || (int)si >= 3 * Dmax)
                                  : (int)si < 3 * Dmax;
      if (in_step) step_bytes += slot_bytes[si];
    }
    if ((int64_t)items.size() > lay.max_items || (int64_t)sweeps.size() > lay.max_sweeps ||
        (int64_t)group_ptrs.size() > 4 * lay.max_sweeps)
      return fail(SLMPP_ERR_WORKSPACE, "batch work lists exceed the workspace");
    hipError_t e = prepare_batch_kernels(dtype, max_lds, max_nxs);
    if (e != hipSuccess) return hip_fail(e, "batch kernel attributes");
    int n_cu = 0, dev = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    for (auto& L : launches) {
      const int per_cu = batch_sweep_blocks_per_cu(dtype, L.lds);
      L.grid = std::max(1, std::min(L.nitems, per_cu * std::max(n_cu, 1)));
    }
    e = hipMemcpyAsync(at<BatchSweep>(lay.sweeps), sweeps.data(), sizeof(BatchSweep) * sweeps.size(),
                       hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !items.empty())
      e = hipMemcpyAsync(at<BatchItem>(lay.items), items.data(), sizeof(BatchItem) * items.size(),
                         hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !group_ptrs.empty())
      e = hipMemcpyAsync(dptrs, group_ptrs.data(), sizeof(void*) * group_ptrs.size(),
                         hipMemcpyHostToDevice, stream);
    mitems2.clear();
    for (int r = 0; r < nruns && !reduce.empty(); ++r)
      if (!mom_fused[r])
        for (int64_t ix = 0; ix < g[r].nxs; ++ix) mitems2.push_back(make_int2(r, (int)ix));
    if (e == hipSuccess && !reduce.empty())
      e = hipMemcpyAsync(at<BatchReduce>(lay.reduce), reduce.data(), sizeof(BatchReduce) * reduce.size(),
                         hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !mitems2.empty())
      e = hipMemcpyAsync(at<int2>(lay.mitems2), mitems2.data(), sizeof(int2) * mitems2.size(),
                         hipMemcpyHostToDevice, stream);
    // the tables of the step's sweeps: x axes (fixed, computed now), v axes
    // (recomputed with the field)
    std::vector<BatchSweep> tl;
    xt_max = vt_max = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int r = 0; r < nruns; ++r)
        for (int l = 0; l < g[r].D; ++l)
          for (int k = 0; k < (pass == 0 ? 1 : (merged ? 2 : 1)); ++k) {
            const SlotDef sd{pass == 1, l, pass == 1 && k == 0 ? 0.5 : 1.0};
            BatchSweep t{};
            int64_t count = 0;
            sweep_of(r, sd, t.a, count);
            t.table = table_of(r, sd);
            t.order = d[r].order;
            t.count = (int32_t)count;
            tl.push_back(t);
            int& mx = pass == 0 ? xt_max : vt_max;
            mx = std::max<int>(mx, (int)count);
          }
    nxt = nvt = 0;
    for (const BatchSweep& t : tl) (t.a.cmode == SPEED_FROM_VELOCITY ? nxt : nvt) += 1;
    if (e == hipSuccess)
      e = hipMemcpyAsync(at<BatchSweep>(lay.tsweeps), tl.data(), sizeof(BatchSweep) * tl.size(),
                         hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_batch_tables(dtype, at<BatchSweep>(lay.tsweeps), nxt, xt_max, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "upload of batch work lists");
    drop_graph();
    return SLMPP_OK;
  }

  void drop_graph() {
    for (int k = 0; k < 4; ++k) {
      if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
      exec[k] = nullptr;
      graph[k] = nullptr;
    }
  }

  hipError_t enqueue_slot(int si, hipStream_t s) {
    const SlotLaunch& L = launches[si];
    if (L.nsweeps == 0) return hipSuccess;
    hipError_t e = hipSuccess;  // the tables were computed at build or with the field
    for (int k = 0; k < L.ngroups && e == hipSuccess; ++k) {
      const FastGroup& fg = groups[(size_t)(L.first_group + k)];
      e = launch_sweep(dtype, fg.order, SLMPP_LIM_MPP, fg.a, fg.p, nullptr, s);
    }
    for (int k = 0; k < L.npgroups && e == hipSuccess; ++k) {
      const PlaneGroup& pg = pgroups[(size_t)(L.first_pgroup + k)];
      e = launch_kick_plane(dtype, pg.order, pg.a, pg.p, nullptr, nullptr, s);
    }
    // (the tile launch after the group launches: run beside them on a
    // second stream it took CU slots from the persistent kernels and made
    // the phase slower)
    if (e == hipSuccess)
      e = launch_batch_sweeps(dtype, at<BatchSweep>(lay.sweeps), at<BatchItem>(lay.items) + L.first_item,
                              L.nitems, L.lds, L.grid, s);
    return e;
  }

  // after_x1: right after the x_1 phase of a step, whose fused groups left
  // row sums; otherwise the moment of every run from f
  hipError_t enqueue_field(hipStream_t s, bool after_x1 = false) {
    hipError_t e;
    if (after_x1 && !reduce.empty()) {
      e = launch_batch_moment(dtype, at<BatchRun>(lay.runs), at<int2>(lay.mitems2), (int)mitems2.size(), s);
      if (e == hipSuccess)
        e = launch_batch_reduce(at<BatchReduce>(lay.reduce), (int)reduce.size(), max_reduce_cells, s);
    } else {
      e = launch_batch_moment(dtype, at<BatchRun>(lay.runs), at<int2>(lay.mitems), (int)lay.nmitems, s);
    }
    if (e == hipSuccess) e = launch_batch_poisson(at<BatchRun>(lay.runs), nruns, max_nxs, s);
    // the velocity sweeps' tables with the new acceleration
    if (e == hipSuccess)
      e = launch_batch_tables(dtype, at<BatchSweep>(lay.tsweeps) + nxt, nvt, vt_max, s);
    return e;
  }

  hipError_t enqueue_range(int first, int count, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int si = first; si < first + count && e == hipSuccess; ++si) e = enqueue_slot(si, s);
    return e;
  }

  // kind: see graph[]
  hipError_t enqueue_kind(int kind, hipStream_t s) {
    const int K = Dmax;
    if (kind == 1) return enqueue_range(0, K, s);
    hipError_t e = kind == 0 ? enqueue_range(0, K, s) : hipSuccess;
    if (e == hipSuccess) e = enqueue_range(K, K, s);
    if (e == hipSuccess) e = enqueue_field(s, true);
    if (e == hipSuccess) e = enqueue_range(kind == 2 ? 3 * K : 2 * K, K, s);
    return e;
  }

  // the kinds of a call of nsteps, in order
  template <typename F>
  hipError_t for_each_kind(int32_t nsteps, F&& run) {
    if (!merged) {
      hipError_t e = hipSuccess;
      for (int32_t i = 0; i < nsteps && e == hipSuccess; ++i) e = run(0);
      return e;
    }
    hipError_t e = run(1);
    for (int32_t i = 0; i + 1 < nsteps && e == hipSuccess; ++i) e = run(2);
    if (e == hipSuccess) e = run(3);
    return e;
  }

  slmpp_status ensure_field() {
    if (field_valid) return SLMPP_OK;
    hipError_t e = enqueue_field(stream);
    if (e != hipSuccess) return hip_fail(e, "batch field");
    field_valid = true;
    return SLMPP_OK;
  }
};

extern "C" {

size_t slmpp_batch_workspace_bytes(const slmpp_grid_desc* descs, int32_t nruns) {
  std::string msg;
  if (check_batch(descs, nruns, msg) != SLMPP_OK) return 0;
  return layout_of(std::vector<slmpp_grid_desc>(descs, descs + nruns)).total;
}

slmpp_status slmpp_batch_create(const slmpp_grid_desc* descs, const double* dts, int32_t nruns,
                                void* const* f_dev, void* work_dev, size_t work_bytes,
                                void* hip_stream, slmpp_batch** out) {
  try {
    if (!out) {
      g_batch_error = "out is NULL";
      return SLMPP_ERR_INVALID;
    }
    *out = nullptr;
    std::string msg;
    slmpp_status st = check_batch(descs, nruns, msg);
    if (st != SLMPP_OK) {
      g_batch_error = msg;
      return st;
    }
    if (!dts || !f_dev || !work_dev) {
      g_batch_error = "dts, f_dev and work_dev must be non-NULL";
      return SLMPP_ERR_INVALID;
    }
    if (reinterpret_cast<uintptr_t>(work_dev) % 256) {
      g_batch_error = "work_dev must be 256-byte aligned";
      return SLMPP_ERR_INVALID;
    }
    for (int r = 0; r < nruns; ++r) {
      if (!std::isfinite(dts[r])) {
        g_batch_error = "dt of run " + std::to_string(r) + " is not finite";
        return SLMPP_ERR_NONFINITE;
      }
      if (!f_dev[r] || reinterpret_cast<uintptr_t>(f_dev[r]) % 16) {
        g_batch_error = "f_dev[" + std::to_string(r) + "] must be non-NULL and 16-byte aligned";
        return SLMPP_ERR_INVALID;
      }
    }
    std::vector<slmpp_grid_desc> dv(descs, descs + nruns);
    Layout lay = layout_of(dv);
    if (work_bytes < lay.total) {
      g_batch_error = "workspace of " + std::to_string(work_bytes) + " bytes, need " +
                      std::to_string(lay.total);
      return SLMPP_ERR_WORKSPACE;
    }
    slmpp_batch* b = new slmpp_batch();
    b->nruns = nruns;
    b->dtype = descs[0].storage;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->d = dv;
    b->dt.assign(dts, dts + nruns);
    b->f.assign(f_dev, f_dev + nruns);
    b->work = static_cast<char*>(work_dev);
    b->work_bytes = work_bytes;
    b->lay = lay;
    std::vector<int2> mitems;
    for (int r = 0; r < nruns; ++r) {
      b->g.push_back(geom_of(dv[r]));
      const RunGeom& G = b->g.back();
      b->Dmax = std::max(b->Dmax, G.D);
      b->max_nxs = std::max<int>(b->max_nxs, (int)G.nxs);
      BatchRun R{};
      R.f = f_dev[r];
      R.rho = b->at<double>(lay.rho[r]);
      R.phi = b->at<double>(lay.phi[r]);
      R.accel = b->at<double>(lay.acc[r]);
      R.nxs = G.nxs;
      R.nvs = G.nvs;
      R.dvol = 1.0;
      for (int l = 0; l < 3; ++l) {
        R.nx[l] = l < G.D ? dv[r].nx[l] : 1;
        R.h[l] = l < G.D ? G.hx[l] : 1.0;
      }
      for (int l = 0; l < G.D; ++l) R.dvol *= G.hv[l];
      R.kappa = dv[r].kappa;
      R.D = G.D;
      R.poisson_order = dv[r].poisson_order;
      b->runs.push_back(R);
      for (int64_t ix = 0; ix < G.nxs; ++ix) mitems.push_back(make_int2(r, (int)ix));
    }
    b->merged = (dv[0].flags & SLMPP_FLAG_MERGE_KICKS) != 0;
    b->slots = slot_defs(b->Dmax, b->merged);
    hipError_t e = hipMemcpyAsync(b->at<BatchRun>(lay.runs), b->runs.data(),
                                  sizeof(BatchRun) * b->runs.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->at<int2>(lay.mitems), mitems.data(), sizeof(int2) * mitems.size(),
                         hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
      g_batch_error = std::string("batch upload: ") + hipGetErrorString(e);
      delete b;
      return SLMPP_ERR_DEVICE;
    }
    st = b->build();
    if (st != SLMPP_OK) {
      g_batch_error = b->err;
      delete b;
      return st;
    }
    *out = b;
    return SLMPP_OK;
  } catch (const std::bad_alloc&) {
    g_batch_error = "host allocation failed";
    return SLMPP_ERR_DEVICE;
  }
}

slmpp_status slmpp_batch_destroy(slmpp_batch* b) {
  if (!b) return SLMPP_ERR_INVALID;
  (void)hipStreamSynchronize(b->stream);
  b->drop_graph();
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
  return SLMPP_OK;
}

const char* slmpp_batch_last_error(const slmpp_batch* b) {
  return b ? b->err.c_str() : g_batch_error.c_str();
}

slmpp_status slmpp_batch_init_separable(slmpp_batch* b, int32_t run, const double* s_host,
                                        const double* g1, const double* g2, const double* g3) {
  if (!b) return SLMPP_ERR_INVALID;
  if (run < 0 || run >= b->nruns) return b->fail(SLMPP_ERR_INVALID, "run index out of range");
  const RunGeom& G = b->g[run];
  const double* gv[3] = {g1, g2, g3};
  if (!s_host) return b->fail(SLMPP_ERR_INVALID, "s_host is NULL");
  for (int l = 0; l < G.D; ++l)
    if (!gv[l]) return b->fail(SLMPP_ERR_INVALID, "a velocity factor is NULL");
  double* st = b->at<double>(b->lay.stage);
  hipError_t e = hipMemcpyAsync(st, s_host, 8 * G.nxs, hipMemcpyHostToDevice, b->stream);
  const double* gd[3] = {nullptr, nullptr, nullptr};
  int64_t off = G.nxs;
  for (int l = 0; l < G.D && e == hipSuccess; ++l) {
    gd[l] = st + off;
    e = hipMemcpyAsync(st + off, gv[l], 8 * b->d[run].nv[l], hipMemcpyHostToDevice, b->stream);
    off += b->d[run].nv[l];
  }
  if (e == hipSuccess)
    e = launch_init_separable(b->dtype, b->f[run], st, gd[0], gd[1], gd[2], G.D, b->d[run].nv,
                              G.nxs, G.nvs, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return b->hip_fail(e, "batch init");
  b->field_valid = false;
  return SLMPP_OK;
}

slmpp_status slmpp_batch_step(slmpp_batch* b, int32_t nsteps) {
  if (!b) return SLMPP_ERR_INVALID;
  if (nsteps < 1) return b->fail(SLMPP_ERR_INVALID, "nsteps must be >= 1");
  slmpp_status st = b->ensure_field();
  if (st != SLMPP_OK) return st;
  // graphs are captured on first use on a private stream (the caller's may
  // be the null stream, which cannot be captured) and replayed on the
  // caller's stream
  const char* what = nullptr;
  hipError_t e = b->for_each_kind(nsteps, [&](int kind) -> hipError_t {
    if (!b->exec[kind]) {
      hipError_t r = hipSuccess;
      if (!b->capture) r = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
      if (r != hipSuccess) {
        what = "capture stream";
        return r;
      }
      r = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed);
      if (r != hipSuccess) {
        what = "begin capture";
        return r;
      }
      const hipError_t el = b->enqueue_kind(kind, b->capture);
      hipGraph_t gr = nullptr;
      r = hipStreamEndCapture(b->capture, &gr);
      if (el != hipSuccess || r != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        what = "step capture";
        return el != hipSuccess ? el : r;
      }
      b->graph[kind] = gr;
      r = hipGraphInstantiate(&b->exec[kind], gr, nullptr, nullptr, 0);
      if (r != hipSuccess) {
        b->drop_graph();
        what = "graph instantiate";
        return r;
      }
    }
    what = "graph launch";
    return hipGraphLaunch(b->exec[kind], b->stream);
  });
  if (e != hipSuccess) return b->hip_fail(e, what ? what : "batch step");
  return SLMPP_OK;
}

slmpp_status slmpp_batch_step_eager(slmpp_batch* b, int32_t nsteps) {
  if (!b) return SLMPP_ERR_INVALID;
  if (nsteps < 1) return b->fail(SLMPP_ERR_INVALID, "nsteps must be >= 1");
  slmpp_status st = b->ensure_field();
  if (st != SLMPP_OK) return st;
  hipError_t e = b->for_each_kind(nsteps, [&](int kind) { return b->enqueue_kind(kind, b->stream); });
  if (e != hipSuccess) return b->hip_fail(e, "batch step");
  return SLMPP_OK;
}

slmpp_status slmpp_batch_get_f(slmpp_batch* b, int32_t run, double* f_host, int64_t n) {
  if (!b) return SLMPP_ERR_INVALID;
  if (run < 0 || run >= b->nruns) return b->fail(SLMPP_ERR_INVALID, "run index out of range");
  if (!f_host) return b->fail(SLMPP_ERR_INVALID, "f_host is NULL");
  if (n != b->g[run].ncell) return b->fail(SLMPP_ERR_SHAPE, "n does not match the run's cells");
  const size_t es = b->dtype == SLMPP_F64 ? 8 : 4;
  const int64_t chunk = b->lay.stage_doubles;
  double* st = b->at<double>(b->lay.stage);
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t m = std::min(chunk, n - off);
    hipError_t e = launch_to_double(b->dtype, static_cast<const char*>(b->f[run]) + off * es, st, m,
                                    b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(f_host + off, st, 8 * m, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "batch get_f");
  }
  return SLMPP_OK;
}

slmpp_status slmpp_batch_autotune(slmpp_batch* b, const char* cache_path) {
  if (!b) return SLMPP_ERR_INVALID;
  // candidates are timed with the runs' real speeds
  slmpp_status st = b->ensure_field();
  if (st != SLMPP_OK) return st;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream is(line);
      std::string dt;
      int order = 0, W = 0;
      int64_t n = 0, inner = 0;
      if (is >> dt >> order >> n >> inner >> W &&
          (W == 128 || W == 64 || W == 32 || W == 16 || W == 8)) {
        const int dtype = dt == "f64" ? SLMPP_F64 : SLMPP_F32;
        b->width[shape_key(dtype, order, n, inner)] = W;
      }
    }
  }
  // one representative sweep per pencil shape not known yet
  struct Rep {
    std::string key;
    int r;
    SweepArgs a;
    int64_t count;
  };
  std::vector<Rep> reps;
  for (size_t si = 0; si < b->slots.size(); ++si)
    for (int r = 0; r < b->nruns; ++r) {
      SweepArgs a;
      int64_t count = 0;
      if (!b->sweep_of(r, b->slots[si], a, count)) continue;
      const std::string key = shape_key(b->dtype, b->d[r].order, a.n, a.inner);
      bool seen = b->width.count(key) > 0;
      for (const Rep& q : reps) seen = seen || q.key == key;
      if (!seen) reps.push_back(Rep{key, r, a, count});
    }
  int n_cu = 1, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return b->fail(SLMPP_ERR_DEVICE, "device query");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return b->fail(SLMPP_ERR_DEVICE, "event create");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return b->fail(SLMPP_ERR_DEVICE, "event create");
  }
  const size_t es = b->dtype == SLMPP_F64 ? 8 : 4;
  const int64_t scratch_elems = (int64_t)(b->lay.stage - b->lay.scratch) / (int64_t)es;
  char* scratch = b->work + b->lay.scratch;
  BatchSweep* dsw = b->at<BatchSweep>(b->lay.sweeps);
  BatchItem* dit = b->at<BatchItem>(b->lay.items);
  std::vector<std::string> fresh;
  std::vector<BatchSweep> hsw;
  std::vector<BatchItem> hit;
  hipError_t e = hipSuccess;
  for (const Rep& q : reps) {
    const int64_t ncell = b->g[q.r].ncell;
    const int64_t tiles8 = (q.a.npen + kMinW - 1) / kMinW;
    // copies of the run: enough tiles to fill the GPU, within the scratch
    // and work-list capacities
    int64_t m = std::max<int64_t>(1, ((int64_t)1 << 22) / ncell);
    m = std::min(m, scratch_elems / ncell);
    m = std::min(m, b->lay.max_sweeps);
    m = std::min(m, b->lay.max_items / std::max<int64_t>(tiles8, 1));
    m = std::max<int64_t>(m, 1);
    e = hipMemcpyAsync(scratch, b->f[q.r], es * ncell, hipMemcpyDeviceToDevice, b->stream);
    for (int64_t k = 1; k < m && e == hipSuccess; k *= 2) {
      const int64_t c = std::min(k, m - k);
      e = hipMemcpyAsync(scratch + es * ncell * k, scratch, es * ncell * c, hipMemcpyDeviceToDevice,
                         b->stream);
    }
    if (e != hipSuccess) break;
    // candidates within the LDS budget when there are any
    std::vector<SweepPlan> cand;
    for (int W : kCandidates) {
      SweepPlan p = plan_batch_sweep(b->dtype, b->d[q.r].order, q.a.n, q.a.npen, q.a.inner,
                                     q.a.nfast, W);
      if (p.lds_bytes && p.lds_bytes <= kBatchTileLds) cand.push_back(p);
    }
    if (cand.empty())
      for (int W : kCandidates) {
        SweepPlan p = plan_batch_sweep(b->dtype, b->d[q.r].order, q.a.n, q.a.npen, q.a.inner,
                                       q.a.nfast, W);
        if (p.lds_bytes) cand.push_back(p);
      }
    int bestW = 0;
    float best = 1e30f;
    for (const SweepPlan& p : cand) {
      hsw.assign((size_t)m, BatchSweep{});
      hit.clear();
      for (int64_t k = 0; k < m; ++k) {
        BatchSweep& w = hsw[(size_t)k];
        w.a = q.a;
        w.a.f = scratch + es * ncell * k;
        w.p = p;
        w.table = b->work + b->lay.tab[q.r];
        w.order = b->d[q.r].order;
        w.count = (int32_t)q.count;
        for (int64_t t = 0; t < p.tiles; ++t) hit.push_back(BatchItem{(int32_t)k, 0, t});
      }
      e = hipMemcpyAsync(dsw, hsw.data(), sizeof(BatchSweep) * hsw.size(), hipMemcpyHostToDevice,
                         b->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dit, hit.data(), sizeof(BatchItem) * hit.size(), hipMemcpyHostToDevice,
                           b->stream);
      if (e == hipSuccess) e = prepare_batch_kernels(b->dtype, p.lds_bytes, b->max_nxs);
      if (e == hipSuccess) e = launch_batch_tables(b->dtype, dsw, 1, (int)q.count, b->stream);
      const int nit = (int)hit.size();
      const int grid =
          std::max(1, std::min(nit, batch_sweep_blocks_per_cu(b->dtype, p.lds_bytes) * n_cu));
      if (e == hipSuccess) e = launch_batch_sweeps(b->dtype, dsw, dit, nit, p.lds_bytes, grid, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
        e = launch_batch_sweeps(b->dtype, dsw, dit, nit, p.lds_bytes, grid, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      if (ms < best) {
        best = ms;
        bestW = p.W;
      }
    }
    if (e != hipSuccess) break;
    if (bestW) {
      b->width[q.key] = bestW;
      fresh.push_back(q.key + " " + std::to_string(bestW));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    b->hip_fail(e, "autotune");
    // the work lists were overwritten: restore them before reporting
    const std::string msg = b->err;
    b->build();
    b->err = msg;
    return SLMPP_ERR_DEVICE;
  }
  if (cache_path && !fresh.empty()) {
    std::ofstream out(cache_path, std::ios::app);
    for (const auto& l : fresh) out << l << '\n';
  }
  return b->build();
}

slmpp_status slmpp_batch_set_fast_min_cells(slmpp_batch* b, int64_t min_cells) {
  if (!b) return SLMPP_ERR_INVALID;
  b->fast_min_cells = min_cells;
  return b->build();
}

double slmpp_batch_step_bytes(const slmpp_batch* b) { return b ? b->step_bytes : 0.0; }

int32_t slmpp_batch_tile_width(const slmpp_batch* b, int32_t run, int32_t axis) {
  if (!b || run < 0 || run >= b->nruns || axis < 0 || axis >= 2 * b->g[run].D) return 0;
  return b->run_axis_width[(size_t)run * 6 + axis];
}

}  // extern "C"
