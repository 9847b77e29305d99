// Host runtime behind the C-ABI of include/slmpp.h: argument validation,
// workspace layout, launch plans, the Strang step and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "slmpp_internal.hpp"

using namespace slmpp;

namespace {

constexpr int64_t kMaxAxis = 4096;               // LDS holds a whole pencil
constexpr int64_t kMaxCells = (int64_t)1 << 40;  // 1.1e12 cells
constexpr int64_t kStageChunk = (int64_t)1 << 22;  // doubles per host<->device chunk

thread_local std::string g_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  size_t rho, phi, accel, green, bufA, bufB, tw, partials, diagfield, table, table2, stage, mom, rkbuf,
      isoA, isoB, isoG, tw2, prun, total;
  int64_t stage_doubles, mom_doubles;
};

int64_t n_space(const slmpp_grid_desc& d) {
  int64_t p = 1;
  for (int l = 0; l < d.D; ++l) p *= d.nx[l];
  return p;
}
int64_t n_vel(const slmpp_grid_desc& d) {
  int64_t p = 1;
  for (int l = 0; l < d.D; ++l) p *= d.nv[l];
  return p;
}

Layout layout_of(const slmpp_grid_desc& d) {
  Layout L{};
  const int64_t nxs = n_space(d), ncell = nxs * n_vel(d);
  int64_t sumnx = 0, sumnv = 0;
  for (int l = 0; l < d.D; ++l) {
    sumnx += d.nx[l];
    sumnv += d.nv[l];
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.rho = take(sizeof(double) * nxs);
  L.phi = take(sizeof(double) * nxs);
  L.accel = take(sizeof(double) * nxs * d.D);
  L.green = take(sizeof(double) * nxs);
  L.bufA = take(sizeof(double2) * nxs);
  L.bufB = take(sizeof(double2) * nxs);
  L.tw = take(sizeof(double2) * sumnx);
  L.partials = take(sizeof(double) * kDiagBlocks * 5);
  L.diagfield = take(sizeof(double) * 4);
  int64_t maxnv = 1;
  for (int l = 0; l < d.D; ++l) maxnv = std::max<int64_t>(maxnv, d.nv[l]);
  L.table = take(pencil_table_bytes(SLMPP_F64, std::max<int64_t>(maxnv, nxs)));
  L.table2 = take(pencil_table_bytes(SLMPP_F64, nxs));  // second axis of a two-axis kick
  L.stage_doubles = std::max<int64_t>(std::min<int64_t>(kStageChunk, ncell), nxs + sumnv);
  L.stage = take(sizeof(double) * L.stage_doubles);
  // row sums of the x_1 sweep's tiles (fused velocity moment; 64 or 128
  // pencils per tile)
  L.mom_doubles = ncell / 64;
  L.mom = take(sizeof(double) * std::max<int64_t>(L.mom_doubles, 1));
  // TVD-RK time integration keeps f^n of a sweep
  L.rkbuf = take((d.flags & SLMPP_FLAG_RK3) ? (size_t)ncell * (d.storage == SLMPP_F64 ? 8 : 4) : 0);
  // isolated boundaries: two complex buffers and the Green transform on the
  // doubled grid, twiddles of the doubled axes
  const bool iso = (d.flags & SLMPP_FLAG_ISOLATED) != 0;
  const int64_t ms = iso ? 8 * nxs : 0;
  L.isoA = take(sizeof(double2) * ms);
  L.isoB = take(sizeof(double2) * ms);
  L.isoG = take(sizeof(double) * ms);
  L.tw2 = take(iso ? sizeof(double2) * 2 * sumnx : 0);
  // small periodic grids: the field of the context in one workgroup
  L.prun = take(sizeof(BatchRun));
  L.total = off;
  return L;
}

bool is_finite(double x) { return std::isfinite(x); }

}  // namespace

slmpp_status slmpp::check_grid_desc(const slmpp_grid_desc* d, std::string& msg) {
  if (!d) {
    msg = "desc is NULL";
    return SLMPP_ERR_INVALID;
  }
  if (d->D < 1 || d->D > 3) {
    msg = "D must be 1, 2 or 3";
    return SLMPP_ERR_INVALID;
  }
  if (d->order != 5 && d->order != 7) {
    msg = "order must be 5 or 7";
    return SLMPP_ERR_INVALID;
  }
  if (d->limiter < SLMPP_LIM_NONE || d->limiter > SLMPP_LIM_MPP) {
    msg = "limiter must be SLMPP_LIM_NONE, SLMPP_LIM_MP or SLMPP_LIM_MPP";
    return SLMPP_ERR_INVALID;
  }
  if (d->poisson_order != 2 && d->poisson_order != 4 && d->poisson_order != 6) {
    msg = "poisson_order must be 2, 4 or 6";
    return SLMPP_ERR_INVALID;
  }
  if (d->storage != SLMPP_F64 && d->storage != SLMPP_F32) {
    msg = "storage must be SLMPP_F64 or SLMPP_F32";
    return SLMPP_ERR_INVALID;
  }
  if ((d->x_bc != SLMPP_BC_PERIODIC && d->x_bc != SLMPP_BC_OUTFLOW) ||
      (d->v_bc != SLMPP_BC_PERIODIC && d->v_bc != SLMPP_BC_OUTFLOW)) {
    msg = "x_bc / v_bc must be SLMPP_BC_PERIODIC or SLMPP_BC_OUTFLOW";
    return SLMPP_ERR_INVALID;
  }
  if ((d->flags & ~(SLMPP_FLAG_RK3 | SLMPP_FLAG_MERGE_KICKS | SLMPP_FLAG_ISOLATED |
                    SLMPP_FLAG_SEPARATE_KICKS)) != 0) {
    msg = "flags must combine SLMPP_FLAG_RK3, SLMPP_FLAG_MERGE_KICKS, SLMPP_FLAG_ISOLATED and "
          "SLMPP_FLAG_SEPARATE_KICKS only";
    return SLMPP_ERR_INVALID;
  }
  if ((d->flags & SLMPP_FLAG_ISOLATED) && d->D != 3) {
    msg = "isolated boundaries need D = 3";
    return SLMPP_ERR_INVALID;
  }
  if (!is_finite(d->alpha) || !(d->alpha > 0.0) || !is_finite(d->kappa)) {
    msg = "alpha must be finite and > 0, kappa finite";
    return SLMPP_ERR_NONFINITE;
  }
  int64_t cells = 1;
  for (int l = 0; l < d->D; ++l) {
    if (d->nx[l] < 1 || d->nx[l] > kMaxAxis || d->nv[l] < 1 || d->nv[l] > kMaxAxis) {
      msg = "every axis needs 1..4096 cells";
      return SLMPP_ERR_SHAPE;
    }
    if (!is_finite(d->x_lo[l]) || !is_finite(d->x_hi[l]) || !is_finite(d->v_lo[l]) ||
        !is_finite(d->v_hi[l])) {
      msg = "domain bounds must be finite";
      return SLMPP_ERR_NONFINITE;
    }
    if (!(d->x_hi[l] > d->x_lo[l]) || !(d->v_hi[l] > d->v_lo[l])) {
      msg = "domain bounds need hi > lo";
      return SLMPP_ERR_SHAPE;
    }
    cells *= d->nx[l];
    cells *= d->nv[l];
    if (cells > kMaxCells) {
      msg = "grid exceeds 2^40 cells";
      return SLMPP_ERR_SHAPE;
    }
  }
  return SLMPP_OK;
}

namespace {
slmpp_status check_desc(const slmpp_grid_desc* d, std::string& msg) { return check_grid_desc(d, msg); }
}  // namespace

namespace {
// The arguments of the sweep along v_l (array axis D + l) of a grid with
// axis sizes dims[0..2D), speed accel[ix] (Eq. (adv_vel)).
SweepArgs v_sweep_args(const slmpp_grid_desc& d, const int64_t* dims, int l, double dt,
                       const double* accel, void* f, int64_t& inner) {
  const int D = d.D, nd = 2 * D, a = D + l;
  inner = 1;
  for (int k = a + 1; k < nd; ++k) inner *= dims[k];
  int64_t outer = 1, xdiv = 1;
  for (int k = 0; k < a; ++k) outer *= dims[k];
  for (int k = D; k < a; ++k) xdiv *= dims[k];
  SweepArgs s{};
  s.f = f;
  s.npen = outer * inner;
  s.inner = inner;
  s.n = (int32_t)dims[a];
  s.dt = dt;
  s.alpha = d.alpha;
  s.cmode = SPEED_FROM_ACCEL;
  s.accel = accel;
  s.xdiv = xdiv;
  s.vdiv = 1;
  s.nvl = 1;
  s.h = (d.v_hi[l] - d.v_lo[l]) / (double)d.nv[l];
  s.bc = d.v_bc;
  s.nfast = 4;
  return s;
}
}  // namespace

struct slmpp_ctx {
  slmpp_grid_desc d{};
  void* f = nullptr;
  char* work = nullptr;
  size_t work_bytes = 0;
  hipStream_t stream = nullptr;
  Layout lay{};
  int D = 1;
  int64_t dims[6]{};
  int64_t nxs = 0, nvs = 0, ncell = 0;
  double hx[3]{}, hv[3]{};
  int64_t tw_off[3]{};
  bool field_valid = false;
  std::string err;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_class;
  std::vector<double> ev_bytes, ev_cells;
  slmpp_timing acc{};

  double* rho() { return reinterpret_cast<double*>(work + lay.rho); }
  double* phi() { return reinterpret_cast<double*>(work + lay.phi); }
  double* accel() { return reinterpret_cast<double*>(work + lay.accel); }
  double* green() { return reinterpret_cast<double*>(work + lay.green); }
  double2* bufA() { return reinterpret_cast<double2*>(work + lay.bufA); }
  double2* bufB() { return reinterpret_cast<double2*>(work + lay.bufB); }
  double2* tw() { return reinterpret_cast<double2*>(work + lay.tw); }
  double* partials() { return reinterpret_cast<double*>(work + lay.partials); }
  double* diagfield() { return reinterpret_cast<double*>(work + lay.diagfield); }
  double* stage() { return reinterpret_cast<double*>(work + lay.stage); }
  void* table() { return work + lay.table; }
  void* table2() { return work + lay.table2; }
  double* mom() { return reinterpret_cast<double*>(work + lay.mom); }
  double2* isoA() { return reinterpret_cast<double2*>(work + lay.isoA); }
  double2* isoB() { return reinterpret_cast<double2*>(work + lay.isoB); }
  double* isoG() { return reinterpret_cast<double*>(work + lay.isoG); }
  double2* tw2() { return reinterpret_cast<double2*>(work + lay.tw2); }
  int64_t tw2_off[3]{};
  bool isolated = false;  // SLMPP_FLAG_ISOLATED
  // periodic grid of at most kBatchMaxSpace cells: the context's own field
  // solve runs as one workgroup in LDS (the batched ensembles' kernel)
  bool small_field = false;
  void* rkbuf() { return work + lay.rkbuf; }
  bool rk = false;  // SLMPP_FLAG_RK3
  int mom_w = 64;  // tile width of the last fused x_1 sweep
  size_t esize() const { return d.storage == SLMPP_F64 ? 8 : 4; }

  slmpp_status fail(slmpp_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  slmpp_status hip_fail(hipError_t e, const char* what) {
    return fail(SLMPP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }

  // --- timing brackets ---
  hipError_t tic(int cls, double bytes, double cells) {
    if (!timing) return hipSuccess;
    while (ev_pool.size() < ev_used + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev_pool.push_back(e);
    }
    ev_class.push_back(cls);
    ev_bytes.push_back(bytes);
    ev_cells.push_back(cells);
    return hipEventRecord(ev_pool[ev_used++], stream);
  }
  hipError_t toc() {
    if (!timing) return hipSuccess;
    return hipEventRecord(ev_pool[ev_used++], stream);
  }
  hipError_t collect() {
    if (ev_used == 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    for (size_t k = 0; k < ev_class.size(); ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev_pool[2 * k], ev_pool[2 * k + 1]);
      if (e != hipSuccess) return e;
      const int c = ev_class[k];
      acc.launches[c] += 1;
      acc.total_ms[c] += ms;
      acc.bytes[c] += ev_bytes[k];
      acc.cells[c] += ev_cells[k];
    }
    ev_used = 0;
    ev_class.clear();
    ev_bytes.clear();
    ev_cells.clear();
    return hipSuccess;
  }

  // TVD-RK needs |v dt / h| <= 1 at every velocity centre of axis l (the
  // end centres bound it)
  slmpp_status check_rk_x(int l, double dt) {
    const double c0 = d.v_lo[l] + 0.5 * hv[l], c1 = d.v_lo[l] + (d.nv[l] - 0.5) * hv[l];
    const double nu = std::max(std::fabs(c0), std::fabs(c1)) * std::fabs(dt) / hx[l];
    if (!(nu <= 1.0))
      return fail(SLMPP_ERR_INVALID, "RK3 time integration needs |v dt / dx| <= 1 (%.3g)", nu);
    return SLMPP_OK;
  }

  // --- one sweep along array axis a ---
  // fuse_moment (x_1 sweeps only): when the sweep runs as strided 64-pencil
  // tiles lying within velocity blocks, it also leaves per-tile row sums for
  // the velocity moment and *fused is set.
  slmpp_status sweep(int a, double dt, const double* accel_dev, bool fuse_moment = false,
                     bool* fused = nullptr) {
    if (fused) *fused = false;
    const int nd = 2 * D;
    int64_t inner = 1;
    for (int k = a + 1; k < nd; ++k) inner *= dims[k];
    int64_t outer = 1;
    for (int k = 0; k < a; ++k) outer *= dims[k];
    SweepArgs s{};
    s.f = f;
    s.npen = outer * inner;
    s.inner = inner;
    s.n = (int32_t)dims[a];
    s.dt = dt;
    s.alpha = d.alpha;
    if (a >= D) {  // v_l sweep, speed a_l(x)
      s = v_sweep_args(d, dims, a - D, dt, accel_dev, f, inner);
    } else {  // x_l sweep, speed v_l
      const int l = a;
      int64_t vdiv = 1;
      for (int k = D + l + 1; k < nd; ++k) vdiv *= dims[k];
      s.cmode = SPEED_FROM_VELOCITY;
      s.vdiv = vdiv;
      s.nvl = (int32_t)d.nv[l];
      s.vlo = d.v_lo[l];
      s.dv = hv[l];
      s.h = hx[l];
      s.bc = d.x_bc;
      s.xdiv = 1;
      s.nfast = max_shift_velocity(s.vlo, s.dv, s.nvl, dt, s.h, s.n, s.bc);
      if (rk) {
        slmpp_status st = check_rk_x(l, dt);
        if (st != SLMPP_OK) return st;
      }
    }
    if (rk) {
      s.rk = 1;
      s.nfast = 0;  // no integer shift in an RK stage
    }
    SweepPlan p = plan_sweep(d.storage, d.order, d.limiter, s.n, s.npen, inner, s.nfast, 0, 0,
                             fuse_moment && !rk && a == 0);
    if (p.lds_bytes > 160 * 1024)
      return fail(SLMPP_ERR_SHAPE, "pencil of %d cells does not fit the LDS tile", s.n);
    if (fuse_moment && !rk && a == 0 && p.fast && p.W >= 64 && inner > 1 &&
        nvs % p.W == 0 && p.tiles * (int64_t)s.n <= lay.mom_doubles) {
      s.mom = mom();
      mom_w = p.W;
      if (fused) *fused = true;
    }
    const double cells = (double)ncell;
    const int64_t tcount = a < D ? d.nv[a] : nxs;
    hipError_t e = tic(5, 0.0, 0.0);
    if (e == hipSuccess) e = launch_pencil_table(d.storage, d.order, s, table(), tcount, stream);
    if (e == hipSuccess) e = toc();
    const int cls = inner == 1 ? 1 : (s.mom ? 6 : (p.W >= 128 ? 0 : 4));
    if (!rk) {
      if (e == hipSuccess) e = tic(cls, 2.0 * cells * esize(), cells);
      if (e == hipSuccess) e = launch_sweep(d.storage, d.order, d.limiter, s, p, table(), stream);
      if (e == hipSuccess) e = toc();
    } else {
      // Eq. (RK): f1 = S(f), f2 = 3/4 f + 1/4 S(f1), f^{n+1} = 1/3 f + 2/3 S(f2),
      // S(u) = u - nu L(u) one stage sweep.  The stages run out of place
      // with the combinations in their stores, f^n staying in f: f1 and f2
      // in rkbuf, the last stage back into f (8 passes over f per sweep)
      if (e == hipSuccess) e = tic(cls, 8.0 * cells * esize(), 3.0 * cells);
      SweepArgs s1 = s, s2 = s, s3 = s;
      s1.fout = rkbuf();
      s2.f = rkbuf();
      s2.fblend = f;
      s2.cb = 0.75;
      s2.cf = 0.25;
      s3.f = rkbuf();
      s3.fout = f;
      s3.fblend = f;
      s3.cb = 1.0 / 3.0;
      s3.cf = 2.0 / 3.0;
      if (e == hipSuccess) e = launch_sweep(d.storage, d.order, d.limiter, s1, p, table(), stream);
      if (e == hipSuccess) e = launch_sweep(d.storage, d.order, d.limiter, s2, p, table(), stream);
      if (e == hipSuccess) e = launch_sweep(d.storage, d.order, d.limiter, s3, p, table(), stream);
      if (e == hipSuccess) e = toc();
    }
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    return SLMPP_OK;
  }

  // The two-axis pass of a kick (v_{D-1}, v_D), when its kernel takes this
  // grid; else lds_bytes == 0.
  PlanePlan kick_plane_plan() const {
    if (D < 2 || rk || d.limiter != SLMPP_LIM_MPP || d.v_bc != SLMPP_BC_OUTFLOW ||
        (d.flags & SLMPP_FLAG_SEPARATE_KICKS))
      return PlanePlan{};
    int64_t vouter = 1;
    for (int l = 0; l < D - 2; ++l) vouter *= d.nv[l];
    return plan_kick_plane(d.storage, d.order, (int32_t)d.nv[D - 2], (int32_t)d.nv[D - 1],
                           nxs * vouter, vouter);
  }

  // The velocity sweeps of one kick, v_1 .. v_D in that order with the
  // current acceleration; v_{D-1} and v_D in one pass when possible.
  slmpp_status kick(double dt) {
    const PlanePlan pp = kick_plane_plan();
    const int nsep = pp.lds_bytes ? D - 2 : D;
    slmpp_status st = SLMPP_OK;
    for (int l = 0; l < nsep && st == SLMPP_OK; ++l) st = sweep(D + l, dt, accel() + (int64_t)l * nxs);
    if (st != SLMPP_OK || nsep == D) return st;
    SweepArgs sa[2];
    for (int k = 0; k < 2; ++k) {
      const int l = D - 2 + k;
      SweepArgs& s = sa[k];
      s = SweepArgs{};
      s.f = f;
      s.n = (int32_t)d.nv[l];
      s.dt = dt;
      s.alpha = d.alpha;
      s.cmode = SPEED_FROM_ACCEL;
      s.accel = accel() + (int64_t)l * nxs;
      s.xdiv = 1;
      s.vdiv = 1;
      s.nvl = 1;
      s.h = hv[l];
      s.bc = d.v_bc;
      s.nfast = 4;
    }
    const double cells = (double)ncell;
    hipError_t e = tic(5, 0.0, 0.0);
    if (e == hipSuccess) e = launch_pencil_table(d.storage, d.order, sa[0], table(), nxs, stream);
    if (e == hipSuccess) e = launch_pencil_table(d.storage, d.order, sa[1], table2(), nxs, stream);
    if (e == hipSuccess) e = toc();
    if (e == hipSuccess) e = tic(7, 2.0 * cells * esize(), 2.0 * cells);
    if (e == hipSuccess) e = launch_kick_plane(d.storage, d.order, sa[0], pp, table(), table2(), stream);
    if (e == hipSuccess) e = toc();
    if (e != hipSuccess) return hip_fail(e, "kick launch");
    return SLMPP_OK;
  }

  slmpp_status moment(double* rho_dev) {
    double dvol = 1.0;
    for (int l = 0; l < D; ++l) dvol *= hv[l];
    hipError_t e = tic(2, (double)ncell * esize() + 8.0 * nxs, 0.0);
    if (e == hipSuccess) e = launch_moment(d.storage, f, nxs, nvs, dvol, rho_dev, stream);
    if (e == hipSuccess) e = toc();
    if (e != hipSuccess) return hip_fail(e, "moment launch");
    return SLMPP_OK;
  }

  slmpp_status poisson(const double* rho_dev, double* phi_dev, double* accel_dev) {
    hipError_t e = tic(3, 8.0 * nxs * (2 + D), 0.0);
    const bool own = rho_dev == rho() && (!phi_dev || phi_dev == phi()) && accel_dev == accel();
    if (e == hipSuccess && small_field && own)
      e = launch_batch_poisson(reinterpret_cast<const BatchRun*>(work + lay.prun), 1, (int)nxs, stream);
    else if (e == hipSuccess && isolated)
      e = launch_poisson_isolated(rho_dev, phi_dev ? phi_dev : phi(), accel_dev, isoA(), isoB(),
                                  tw2(), tw2_off, isoG(), d.nx, hx, d.poisson_order, stream);
    else if (e == hipSuccess)
      e = launch_poisson(rho_dev, phi_dev ? phi_dev : phi(), accel_dev, bufA(), bufB(), tw(),
                         tw_off, green(), D, d.nx, hx, d.poisson_order, stream);
    if (e == hipSuccess) e = toc();
    if (e != hipSuccess) return hip_fail(e, "poisson launch");
    return SLMPP_OK;
  }

  // one Strang step with the current field: kick, x sweeps, field, kick
  slmpp_status step_body(double dt) {
    slmpp_status st = kick(0.5 * dt);
    bool fused = false;
    for (int l = D - 1; l >= 0 && st == SLMPP_OK; --l) st = sweep(l, dt, nullptr, l == 0, &fused);
    if (st == SLMPP_OK) st = fused ? field_from_rowsums() : field();
    if (st == SLMPP_OK) st = kick(0.5 * dt);
    return st;
  }

  // the field after an x_1 sweep that left its tile row sums (see sweep)
  slmpp_status field_from_rowsums() {
    double dvol = 1.0;
    for (int l = 0; l < D; ++l) dvol *= hv[l];
    const int n = (int)d.nx[0];
    const int64_t ncol = nxs / n, nsub = nvs / mom_w;
    hipError_t e = tic(2, 8.0 * (double)ncol * nsub * n + 8.0 * nxs, 0.0);
    if (e == hipSuccess) e = launch_moment_reduce(mom(), n, ncol, nsub, dvol, rho(), stream);
    if (e == hipSuccess) e = toc();
    if (e != hipSuccess) return hip_fail(e, "moment reduce launch");
    slmpp_status st = poisson(rho(), phi(), accel());
    if (st == SLMPP_OK) field_valid = true;
    return st;
  }

  slmpp_status field() {
    slmpp_status st = moment(rho());
    if (st == SLMPP_OK) st = poisson(rho(), phi(), accel());
    if (st == SLMPP_OK) field_valid = true;
    return st;
  }
};

namespace {

// Laplacian symbol times Delta^2 of the 2nd/4th/6th-order stencils of
// App. C (sum of one-dimensional symbols for several axes).
double lap_symbol(double th, int order) {
  const double a = std::sin(0.5 * th), b = std::sin(th), c = std::sin(1.5 * th);
  if (order == 2) return -4.0 * a * a;
  if (order == 4) return (b * b - 16.0 * a * a) / 3.0;
  return (-2.0 * c * c + 27.0 * b * b - 270.0 * a * a) / 45.0;
}

slmpp_status sync_status(slmpp_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "stream synchronize");
  return SLMPP_OK;
}

}  // namespace

namespace {
// Device memory of slmpp_advect_v_noalloc: one pencil table, in a
// file-scope array that every GPU the library runs on holds until the
// process ends (no allocation call).  Host code never uses the array's
// name as an address: each device's copy is looked up once with
// hipGetSymbolAddress and kept per device.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_dev[kMaxDevices] = {};

hipError_t scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

int32_t slmpp_abi_version(void) { return SLMPP_ABI_VERSION; }

size_t slmpp_workspace_bytes(const slmpp_grid_desc* desc) {
  std::string msg;
  if (check_desc(desc, msg) != SLMPP_OK) return 0;
  return layout_of(*desc).total;
}

slmpp_status slmpp_validate(const slmpp_grid_desc* desc, char* msg, size_t msg_len) {
  std::string m;
  slmpp_status st = check_desc(desc, m);
  if (msg && msg_len) {
    std::snprintf(msg, msg_len, "%s", m.c_str());
  }
  if (st != SLMPP_OK) g_error = m;
  return st;
}

namespace {
// Integral of 1/r over the box [-a, a] x [-b, b] x [-c, c]: eight octants
// with the closed form of the potential of a uniform box at its centre.
double box_inverse_r(double a, double b, double c) {
  const double r = std::sqrt(a * a + b * b + c * c);
  double v = b * c * std::asinh(a / std::sqrt(b * b + c * c));
  v += a * c * std::asinh(b / std::sqrt(a * a + c * c));
  v += a * b * std::asinh(c / std::sqrt(a * a + b * b));
  v -= 0.5 * a * a * std::atan(b * c / (a * r));
  v -= 0.5 * b * b * std::atan(a * c / (b * r));
  v -= 0.5 * c * c * std::atan(a * b / (c * r));
  return 8.0 * v;
}
}  // namespace

// Isolated boundaries, doubling-up method (Sec. 2.2): the Green function
// -kappa / (4 pi r) times the cell volume at the minimum-image separations
// of the doubled grid (the cell mean of 1/r at r = 0), transformed once.
hipError_t iso_setup(slmpp_ctx* c, const slmpp_grid_desc& d) {
  const int64_t m[3] = {2 * d.nx[0], 2 * d.nx[1], 2 * d.nx[2]};
  const int64_t ms = m[0] * m[1] * m[2];
  const double h[3] = {c->hx[0], c->hx[1], c->hx[2]};
  const double vol = h[0] * h[1] * h[2];
  const double self = box_inverse_r(0.5 * h[0], 0.5 * h[1], 0.5 * h[2]) / vol;
  std::vector<double2> g(ms);
  for (int64_t i = 0; i < m[0]; ++i)
    for (int64_t j = 0; j < m[1]; ++j)
      for (int64_t k = 0; k < m[2]; ++k) {
        const double dx = (double)(i < d.nx[0] ? i : i - m[0]) * h[0];
        const double dy = (double)(j < d.nx[1] ? j : j - m[1]) * h[1];
        const double dz = (double)(k < d.nx[2] ? k : k - m[2]) * h[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double inv_r = r2 > 0.0 ? 1.0 / std::sqrt(r2) : self;
        g[(i * m[1] + j) * m[2] + k] = make_double2(-d.kappa / (4.0 * M_PI) * inv_r * vol, 0.0);
      }
  std::vector<double2> tw;
  for (int l = 0; l < 3; ++l) {
    c->tw2_off[l] = (int64_t)tw.size();
    for (int64_t q = 0; q < m[l]; ++q) {
      const double ang = 2.0 * M_PI * (double)q / (double)m[l];
      tw.push_back(make_double2(std::cos(ang), -std::sin(ang)));
    }
  }
  hipError_t e = hipMemcpyAsync(c->isoA(), g.data(), sizeof(double2) * ms, hipMemcpyHostToDevice,
                                c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->tw2(), tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = launch_iso_green(c->isoA(), c->isoB(), c->tw2(), c->tw2_off, m, c->isoG(),
                                            c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}

slmpp_status slmpp_create(const slmpp_grid_desc* desc, void* f_dev, void* work_dev,
                          size_t work_bytes, void* hip_stream, slmpp_ctx** out) {
  try {
    std::string msg;
    if (!out) {
      g_error = "out is NULL";
      return SLMPP_ERR_INVALID;
    }
    *out = nullptr;
    slmpp_status st = check_desc(desc, msg);
    if (st != SLMPP_OK) {
      g_error = msg;
      return st;
    }
    if (!f_dev || !work_dev) {
      g_error = "f_dev and work_dev must be non-NULL";
      return SLMPP_ERR_INVALID;
    }
    if (reinterpret_cast<uintptr_t>(work_dev) % 256 != 0 ||
        reinterpret_cast<uintptr_t>(f_dev) % 16 != 0) {
      g_error = "work_dev must be 256-byte and f_dev 16-byte aligned";
      return SLMPP_ERR_INVALID;
    }
    Layout lay = layout_of(*desc);
    if (work_bytes < lay.total) {
      g_error = "workspace of " + std::to_string(work_bytes) + " bytes, need " +
                std::to_string(lay.total);
      return SLMPP_ERR_WORKSPACE;
    }
    slmpp_ctx* c = new slmpp_ctx();
    c->d = *desc;
    c->f = f_dev;
    c->work = static_cast<char*>(work_dev);
    c->work_bytes = work_bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->lay = lay;
    c->D = desc->D;
    c->rk = (desc->flags & SLMPP_FLAG_RK3) != 0;
    for (int l = 0; l < c->D; ++l) {
      c->dims[l] = desc->nx[l];
      c->dims[c->D + l] = desc->nv[l];
      c->hx[l] = (desc->x_hi[l] - desc->x_lo[l]) / (double)desc->nx[l];
      c->hv[l] = (desc->v_hi[l] - desc->v_lo[l]) / (double)desc->nv[l];
    }
    c->nxs = n_space(*desc);
    c->nvs = n_vel(*desc);
    c->ncell = c->nxs * c->nvs;
    // Green function table and twiddles
    std::vector<double> green(c->nxs);
    for (int64_t idx = 0; idx < c->nxs; ++idx) {
      int64_t rem = idx;
      int64_t k[3] = {0, 0, 0};
      for (int l = c->D - 1; l >= 0; --l) {
        k[l] = rem % desc->nx[l];
        rem /= desc->nx[l];
      }
      double L = 0.0;
      bool zero = true;
      for (int l = 0; l < c->D; ++l) {
        if (k[l]) zero = false;
        const double th = 2.0 * M_PI * (double)k[l] / (double)desc->nx[l];
        L += lap_symbol(th, desc->poisson_order) / (c->hx[l] * c->hx[l]);
      }
      green[idx] = zero ? 0.0 : desc->kappa / L;
    }
    std::vector<double2> tw;
    for (int l = 0; l < c->D; ++l) {
      c->tw_off[l] = (int64_t)tw.size();
      for (int64_t q = 0; q < desc->nx[l]; ++q) {
        const double ang = 2.0 * M_PI * (double)q / (double)desc->nx[l];
        tw.push_back(make_double2(std::cos(ang), -std::sin(ang)));
      }
    }
    hipError_t e = hipMemcpyAsync(c->green(), green.data(), sizeof(double) * green.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->tw(), tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->isolated = (desc->flags & SLMPP_FLAG_ISOLATED) != 0;
    if (e == hipSuccess && c->isolated) e = iso_setup(c, *desc);
    if (e == hipSuccess && !c->isolated && c->nxs <= kBatchMaxSpace) {
      BatchRun R{};
      R.f = c->f;
      R.rho = c->rho();
      R.phi = c->phi();
      R.accel = c->accel();
      R.nxs = c->nxs;
      R.nvs = c->nvs;
      R.dvol = 1.0;
      for (int l = 0; l < 3; ++l) {
        R.nx[l] = l < c->D ? desc->nx[l] : 1;
        R.h[l] = l < c->D ? c->hx[l] : 1.0;
      }
      R.kappa = desc->kappa;
      R.D = c->D;
      R.poisson_order = desc->poisson_order;
      e = hipMemcpyAsync(c->work + c->lay.prun, &R, sizeof(R), hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = prepare_batch_kernels(desc->storage, 0, (int)c->nxs);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      c->small_field = e == hipSuccess;
    }
    if (e != hipSuccess) {
      g_error = std::string("upload of field tables: ") + hipGetErrorString(e);
      delete c;
      return SLMPP_ERR_DEVICE;
    }
    *out = c;
    return SLMPP_OK;
  } catch (const std::bad_alloc&) {
    g_error = "host allocation failed";
    return SLMPP_ERR_DEVICE;
  }
}

slmpp_status slmpp_destroy(slmpp_ctx* ctx) {
  if (!ctx) return SLMPP_ERR_INVALID;
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return SLMPP_OK;
}

const char* slmpp_last_error(const slmpp_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_error.c_str();
}

slmpp_status slmpp_init_f_host(slmpp_ctx* c, const double* f_host, int64_t n) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!f_host) return c->fail(SLMPP_ERR_INVALID, "f_host is NULL");
  if (n != c->ncell) return c->fail(SLMPP_ERR_SHAPE, "n = %lld, grid has %lld cells", (long long)n, (long long)c->ncell);
  const int64_t chunk = c->lay.stage_doubles;
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t m = std::min(chunk, n - off);
    hipError_t e = hipMemcpyAsync(c->stage(), f_host + off, sizeof(double) * m,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = launch_from_double(c->d.storage, static_cast<char*>(c->f) + off * c->esize(), c->stage(), m,
                             c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "init_f_host");
  }
  c->field_valid = false;
  return SLMPP_OK;
}

slmpp_status slmpp_init_f_separable(slmpp_ctx* c, const double* s_host, const double* g1,
                                    const double* g2, const double* g3) {
  if (!c) return SLMPP_ERR_INVALID;
  const double* g[3] = {g1, g2, g3};
  if (!s_host) return c->fail(SLMPP_ERR_INVALID, "s_host is NULL");
  for (int l = 0; l < c->D; ++l)
    if (!g[l]) return c->fail(SLMPP_ERR_INVALID, "velocity factor %d is NULL", l + 1);
  double* st = c->stage();
  hipError_t e = hipMemcpyAsync(st, s_host, sizeof(double) * c->nxs, hipMemcpyHostToDevice, c->stream);
  const double* gd[3] = {nullptr, nullptr, nullptr};
  int64_t off = c->nxs;
  for (int l = 0; l < c->D && e == hipSuccess; ++l) {
    gd[l] = st + off;
    e = hipMemcpyAsync(st + off, g[l], sizeof(double) * c->d.nv[l], hipMemcpyHostToDevice, c->stream);
    off += c->d.nv[l];
  }
  if (e == hipSuccess)
    e = launch_init_separable(c->d.storage, c->f, st, gd[0], gd[1], gd[2], c->D, c->d.nv, c->nxs,
                              c->nvs, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "init_f_separable");
  c->field_valid = false;
  return SLMPP_OK;
}

slmpp_status slmpp_advect_x(slmpp_ctx* c, int32_t dim, double dt) {
  if (!c) return SLMPP_ERR_INVALID;
  if (dim < 0 || dim >= c->D) return c->fail(SLMPP_ERR_INVALID, "dim %d outside 0..%d", dim, c->D - 1);
  if (!std::isfinite(dt)) return c->fail(SLMPP_ERR_NONFINITE, "dt is not finite");
  c->field_valid = false;
  if (dt == 0.0) return SLMPP_OK;
  return c->sweep(dim, dt, nullptr);
}

slmpp_status slmpp_advect_v(slmpp_ctx* c, int32_t dim, double dt, const double* accel_dev) {
  if (!c) return SLMPP_ERR_INVALID;
  if (dim < 0 || dim >= c->D) return c->fail(SLMPP_ERR_INVALID, "dim %d outside 0..%d", dim, c->D - 1);
  if (!std::isfinite(dt)) return c->fail(SLMPP_ERR_NONFINITE, "dt is not finite");
  if (!accel_dev) return c->fail(SLMPP_ERR_INVALID, "accel_dev is NULL");
  c->field_valid = false;
  if (dt == 0.0) return SLMPP_OK;
  return c->sweep(c->D + dim, dt, accel_dev);
}

slmpp_status slmpp_advect_v_noalloc(const slmpp_grid_desc* desc, void* f_dev, int32_t dim,
                                    double dt, const double* accel_dev, void* hip_stream) {
  std::string msg;
  slmpp_status st = check_desc(desc, msg);
  if (st != SLMPP_OK) {
    g_error = msg;
    return st;
  }
  if (!f_dev || !accel_dev) {
    g_error = "f_dev and accel_dev must be non-NULL";
    return SLMPP_ERR_INVALID;
  }
  if (reinterpret_cast<uintptr_t>(f_dev) % 16 != 0) {
    g_error = "f_dev must be 16-byte aligned";
    return SLMPP_ERR_INVALID;
  }
  if (dim < 0 || dim >= desc->D) {
    g_error = "dim " + std::to_string(dim) + " outside 0.." + std::to_string(desc->D - 1);
    return SLMPP_ERR_INVALID;
  }
  if (!std::isfinite(dt)) {
    g_error = "dt is not finite";
    return SLMPP_ERR_NONFINITE;
  }
  if (desc->flags & SLMPP_FLAG_RK3) {
    g_error = "RK3 time integration needs a workspace copy of f: use slmpp_advect_v";
    return SLMPP_ERR_INVALID;
  }
  const int D = desc->D;
  int64_t dims[6];
  for (int l = 0; l < D; ++l) {
    dims[l] = desc->nx[l];
    dims[D + l] = desc->nv[l];
  }
  const int64_t nxs = n_space(*desc);
  const size_t need = pencil_table_bytes(desc->storage, nxs);
  if (need > kNoAllocScratchBytes) {
    g_error = "velocity sweep of " + std::to_string(nxs) + " spatial cells needs " +
              std::to_string(need) + " bytes of scratch; the limit is " +
              std::to_string(kNoAllocScratchBytes) + " (use slmpp_advect_v)";
    return SLMPP_ERR_SHAPE;
  }
  if (dt == 0.0) return SLMPP_OK;
  int64_t inner = 1;
  const SweepArgs s = v_sweep_args(*desc, dims, dim, dt, accel_dev, f_dev, inner);
  const SweepPlan p = plan_sweep(desc->storage, desc->order, desc->limiter, s.n, s.npen, inner,
                                 s.nfast);
  if (p.lds_bytes > 160 * 1024) {
    g_error = "pencil of " + std::to_string(s.n) + " cells does not fit the LDS tile";
    return SLMPP_ERR_SHAPE;
  }
  void* table = nullptr;
  hipError_t e = scratch_for_current_device(&table);
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  if (e == hipSuccess) e = launch_pencil_table(desc->storage, desc->order, s, table, nxs, stream);
  if (e == hipSuccess) e = launch_sweep(desc->storage, desc->order, desc->limiter, s, p, table, stream);
  if (e != hipSuccess) {
    g_error = std::string("advect_v_noalloc: ") + hipGetErrorString(e);
    return SLMPP_ERR_DEVICE;
  }
  return SLMPP_OK;
}

slmpp_status slmpp_kick(slmpp_ctx* c, double dt) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!std::isfinite(dt)) return c->fail(SLMPP_ERR_NONFINITE, "dt is not finite");
  slmpp_status st = SLMPP_OK;
  if (!c->field_valid) st = c->field();
  if (st != SLMPP_OK || dt == 0.0) return st;
  c->field_valid = false;
  return c->kick(dt);
}

slmpp_status slmpp_density_moment(slmpp_ctx* c, double* rho_dev) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!rho_dev) return c->fail(SLMPP_ERR_INVALID, "rho_dev is NULL");
  return c->moment(rho_dev);
}

slmpp_status slmpp_velocity_moments(slmpp_ctx* c, double* rho_dev, double* mean_dev,
                                    double* disp_dev) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!rho_dev || !mean_dev || !disp_dev)
    return c->fail(SLMPP_ERR_INVALID, "rho_dev, mean_dev and disp_dev must be non-NULL");
  hipError_t e = launch_velocity_moments(c->d.storage, c->f, c->D, c->d.nv, c->d.v_lo, c->hv,
                                         c->nxs, rho_dev, mean_dev, disp_dev, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "velocity moments launch");
  return SLMPP_OK;
}

slmpp_status slmpp_velocity_distribution(slmpp_ctx* c, double* F_dev) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!F_dev) return c->fail(SLMPP_ERR_INVALID, "F_dev is NULL");
  double xvol = 1.0;
  for (int l = 0; l < c->D; ++l) xvol *= c->hx[l];
  hipError_t e = launch_velocity_distribution(c->d.storage, c->f, c->nxs, c->nvs, xvol, F_dev,
                                              c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "velocity distribution launch");
  return SLMPP_OK;
}

slmpp_status slmpp_poisson_solve(slmpp_ctx* c, const double* rho_dev, double* phi_dev,
                                 double* accel_dev) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!rho_dev || !accel_dev) return c->fail(SLMPP_ERR_INVALID, "rho_dev and accel_dev must be non-NULL");
  return c->poisson(rho_dev, phi_dev, accel_dev);
}

slmpp_status slmpp_field(slmpp_ctx* c) {
  if (!c) return SLMPP_ERR_INVALID;
  return c->field();
}

slmpp_status slmpp_field_ptrs(const slmpp_ctx* cc, const double** rho_dev, const double** phi_dev,
                              const double** accel_dev) {
  if (!cc) return SLMPP_ERR_INVALID;
  slmpp_ctx* c = const_cast<slmpp_ctx*>(cc);
  if (rho_dev) *rho_dev = c->rho();
  if (phi_dev) *phi_dev = c->phi();
  if (accel_dev) *accel_dev = c->accel();
  return SLMPP_OK;
}

slmpp_status slmpp_get_field(slmpp_ctx* c, double* rho_host, double* accel_host) {
  if (!c) return SLMPP_ERR_INVALID;
  hipError_t e = hipSuccess;
  if (rho_host)
    e = hipMemcpyAsync(rho_host, c->rho(), sizeof(double) * c->nxs, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && accel_host)
    e = hipMemcpyAsync(accel_host, c->accel(), sizeof(double) * c->nxs * c->D,
                       hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "get_field");
  return SLMPP_OK;
}

slmpp_status slmpp_step(slmpp_ctx* c, double dt, int32_t nsteps) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!std::isfinite(dt)) return c->fail(SLMPP_ERR_NONFINITE, "dt is not finite");
  if (nsteps < 1) return c->fail(SLMPP_ERR_INVALID, "nsteps must be >= 1");
  const int D = c->D;
  if (c->rk) {  // refuse before any work
    for (int l = 0; l < D; ++l) {
      slmpp_status st = c->check_rk_x(l, dt);
      if (st != SLMPP_OK) return st;
    }
  }
  if (c->d.flags & SLMPP_FLAG_MERGE_KICKS) {
    // v(dt/2) [x block, field, v(dt)]... ending with v(dt/2)
    slmpp_status st = SLMPP_OK;
    if (!c->field_valid) st = c->field();
    if (st == SLMPP_OK) st = c->kick(0.5 * dt);
    for (int32_t it = 0; it < nsteps && st == SLMPP_OK; ++it) {
      bool fused = false;
      for (int l = D - 1; l >= 0 && st == SLMPP_OK; --l)
        st = c->sweep(l, dt, nullptr, l == 0, &fused);
      if (st == SLMPP_OK) st = fused ? c->field_from_rowsums() : c->field();
      if (st == SLMPP_OK) st = c->kick(it + 1 < nsteps ? dt : 0.5 * dt);
    }
    if (st != SLMPP_OK) c->field_valid = false;
    return st;
  }
  for (int32_t it = 0; it < nsteps; ++it) {
    slmpp_status st = SLMPP_OK;
    if (!c->field_valid) st = c->field();
    if (st == SLMPP_OK) st = c->step_body(dt);
    if (st != SLMPP_OK) {
      c->field_valid = false;
      return st;
    }
  }
  return SLMPP_OK;
}

slmpp_status slmpp_get_f(slmpp_ctx* c, double* f_host, int64_t n) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!f_host) return c->fail(SLMPP_ERR_INVALID, "f_host is NULL");
  if (n != c->ncell) return c->fail(SLMPP_ERR_SHAPE, "n = %lld, grid has %lld cells", (long long)n, (long long)c->ncell);
  const int64_t chunk = c->lay.stage_doubles;
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t m = std::min(chunk, n - off);
    hipError_t e = launch_to_double(c->d.storage, static_cast<const char*>(c->f) + off * c->esize(),
                                    c->stage(), m, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(f_host + off, c->stage(), sizeof(double) * m, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "get_f");
  }
  return SLMPP_OK;
}

slmpp_status slmpp_diag(slmpp_ctx* c, slmpp_diag_out* out) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!out) return c->fail(SLMPP_ERR_INVALID, "out is NULL");
  slmpp_status st = SLMPP_OK;
  if (!c->field_valid) st = c->field();
  if (st != SLMPP_OK) return st;
  const int nb = kDiagBlocks;
  hipError_t e = launch_diag_f(c->d.storage, c->f, c->ncell, c->partials(), nb, c->stream);
  int64_t inner1 = 1;
  for (int l = 1; l < c->D; ++l) inner1 *= c->d.nx[l];
  if (e == hipSuccess)
    e = launch_diag_field(c->accel(), c->D, c->nxs, c->d.nx[0], inner1, c->diagfield(), c->stream);
  std::vector<double> part(nb * 5);
  double fld[3];
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), c->partials(), sizeof(double) * nb * 5, hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(fld, c->diagfield(), sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "diag");
  double s = 0.0, comp = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double x = part[b * 4 + 0];
    const double t = s + x;
    comp += (std::fabs(s) >= std::fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
    comp += part[b * 4 + 1];
    mn = std::min(mn, part[b * 4 + 2]);
    mx = std::max(mx, part[b * 4 + 3]);
    bad += part[nb * 4 + b];
  }
  double vol = 1.0, dxv = 1.0;
  for (int l = 0; l < c->D; ++l) {
    vol *= c->hx[l] * c->hv[l];
    dxv *= c->hx[l];
  }
  out->mass = vol * (s + comp);
  out->f_min = mn;
  out->f_max = mx;
  out->nonfinite = (int64_t)bad;
  out->field_energy = 0.5 * fld[0] * dxv;
  out->mode_amp = std::sqrt(fld[1] * fld[1] + fld[2] * fld[2]) / (double)c->nxs;
  return SLMPP_OK;
}

slmpp_status slmpp_sync(slmpp_ctx* c) {
  if (!c) return SLMPP_ERR_INVALID;
  return sync_status(c);
}

slmpp_status slmpp_timing_enable(slmpp_ctx* c, int32_t on) {
  if (!c) return SLMPP_ERR_INVALID;
  hipError_t e = c->collect();
  if (e != hipSuccess) return c->hip_fail(e, "timing");
  c->timing = on != 0;
  c->acc = slmpp_timing{};
  return SLMPP_OK;
}

slmpp_status slmpp_timing_read(slmpp_ctx* c, slmpp_timing* out) {
  if (!c) return SLMPP_ERR_INVALID;
  if (!out) return c->fail(SLMPP_ERR_INVALID, "out is NULL");
  hipError_t e = c->collect();
  if (e != hipSuccess) return c->hip_fail(e, "timing");
  *out = c->acc;
  return SLMPP_OK;
}

slmpp_status slmpp_copy_device(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream) {
  if (!dst_dev || !src_dev) {
    g_error = "copy: NULL pointer";
    return SLMPP_ERR_INVALID;
  }
  if (reinterpret_cast<uintptr_t>(dst_dev) % 16 || reinterpret_cast<uintptr_t>(src_dev) % 16 ||
      bytes % 16) {
    g_error = "copy: pointers and size must be multiples of 16 bytes";
    return SLMPP_ERR_INVALID;
  }
  hipError_t e = launch_copy(dst_dev, src_dev, bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) {
    g_error = std::string("copy: ") + hipGetErrorString(e);
    return SLMPP_ERR_DEVICE;
  }
  return SLMPP_OK;
}

slmpp_status slmpp_alloc_device(size_t bytes, int32_t contiguous, void** out) {
  if (out) *out = nullptr;
  if (!out || bytes == 0) {
    g_error = "alloc_device: out is NULL or bytes is 0";
    return SLMPP_ERR_INVALID;
  }
  void* p = nullptr;
  const hipError_t e = contiguous ? hipExtMallocWithFlags(&p, bytes, hipDeviceMallocContiguous)
                                  : hipMalloc(&p, bytes);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();  // the failed allocation's error is reported here, not by the next call
    g_error = std::string("alloc_device: ") + std::to_string(bytes) + " bytes" +
              (contiguous ? " of contiguous memory" : "") + ": " + hipGetErrorString(e);
    return SLMPP_ERR_DEVICE;
  }
  *out = p;
  return SLMPP_OK;
}

slmpp_status slmpp_free_device(void* p) {
  if (!p) return SLMPP_OK;
  const hipError_t e = hipFree(p);
  if (e != hipSuccess) {
    g_error = std::string("free_device: ") + hipGetErrorString(e);
    return SLMPP_ERR_DEVICE;
  }
  return SLMPP_OK;
}

}  // extern "C"
