// Fused SL-MPP sweep kernels for gfx950.
//
// One launch advances every pencil along one axis of f by one
// semi-Lagrangian step (Sec. 2.1.2, Eq. (SL)):
//   xi = c dt / h  ->  integer shift N = floor(xi + 1/2), zeta = xi - N
//   Phi_{i-1/2}    =  CSL5 / CSL7 polynomial in zeta (rows C_j / D_j)
//   Phibar         =  MP constraint (App. A) on the 5-point stencil
//   Phihat         =  PP flux limiter (Sec. 2.1.1)
//   f_i^{n+1}      =  f_{i-N} - zeta (Phihat_{i+1/2} - Phihat_{i-1/2})
// For zeta < 0 the shifted pencil is processed in reverse order, which is
// the mirror image of the c > 0 construction the paper writes out.
//
// Data movement: a workgroup owns a tile of W whole pencils.  It streams
// the tile from HBM into LDS once (coalesced along the contiguous axis,
// whichever way the pencils run), fills ghost rows (periodic images or
// zeros), computes every pencil from LDS with a register sliding window
// (each interface flux is computed once and reused by both neighbouring
// cells), stages the results in LDS and streams them back in place.  So a
// sweep costs one HBM read and one HBM write of f; stencil halos never
// leave the chip.  The same kernel serves strided axes (a tile row is W
// consecutive elements) and the contiguous axis (a tile is W consecutive
// pencils, transposed through LDS); the LDS row pitch W+1 keeps both the
// staging writes and the per-pencil reads free of bank conflicts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "slmpp_internal.hpp"

namespace slmpp {
namespace {

enum : int32_t { READ_DIRECT = 0, READ_WRAP = 1, READ_CLAMP = 2 };

template <typename T>
struct alignas(8) ColParam {
  T w[7];        // FIR weights of the CSL flux at |zeta|
  T z;           // |zeta|
  int32_t base;  // physical row read at processing position 0 (before wrap)
  int32_t dir;   // +1 forward, -1 mirrored (zeta < 0)
  int32_t mode;  // READ_*
  int32_t valid;
};

// CSL flux as an FIR filter: Phi_{i-1/2} = sum_k w_k(zeta) f_{i-h+k} with
// h = 3 (fifth order) or 4 (seventh order), w_k(zeta) = sum_j K[k][j] zeta^j.
// K is the transpose of the coefficient rows C_0..C_4 (D_0..D_6) of
// Sec. 2.1.2, each entry a numerator over the row's common denominator.
struct Frac {
  double num, den;
};
__device__ constexpr Frac kCsl5[5][5] = {
    // zeta^0      zeta^1       zeta^2       zeta^3       zeta^4
    {{2, 60}, {0, 24}, {-1, 24}, {0, 24}, {1, 120}},      // f_{i-3}
    {{-13, 60}, {-1, 24}, {6, 24}, {1, 24}, {-4, 120}},   // f_{i-2}
    {{47, 60}, {15, 24}, {-8, 24}, {-3, 24}, {6, 120}},   // f_{i-1}
    {{27, 60}, {-15, 24}, {2, 24}, {3, 24}, {-4, 120}},   // f_i
    {{-3, 60}, {1, 24}, {1, 24}, {-1, 24}, {1, 120}},     // f_{i+1}
};
__device__ constexpr Frac kCsl7[7][7] = {
    {{-3, 420}, {0, 360}, {7, 720}, {0, 144}, {-2, 720}, {0, 720}, {1, 5040}},        // f_{i-4}
    {{25, 420}, {2, 360}, {-57, 720}, {-1, 144}, {15, 720}, {1, 720}, {-6, 5040}},    // f_{i-3}
    {{-101, 420}, {-25, 360}, {210, 720}, {11, 144}, {-39, 720}, {-5, 720}, {15, 5040}},  // f_{i-2}
    {{319, 420}, {245, 360}, {-230, 720}, {-28, 144}, {46, 720}, {10, 720}, {-20, 5040}}, // f_{i-1}
    {{214, 420}, {-245, 360}, {15, 720}, {28, 144}, {-24, 720}, {-10, 720}, {15, 5040}},  // f_i
    {{-38, 420}, {25, 360}, {63, 720}, {-11, 144}, {3, 720}, {5, 720}, {-6, 5040}},   // f_{i+1}
    {{4, 420}, {-2, 360}, {-8, 720}, {1, 144}, {1, 720}, {-1, 720}, {1, 5040}},       // f_{i+2}
};

// Cell centre and departure offset with the rounding fixed (no FMA
// contraction), so that the integer split agrees with any other IEEE
// evaluation of the same expressions.
__device__ __forceinline__ double cell_center(double lo, double d, int64_t j) {
#pragma clang fp contract(off)
  return lo + ((double)j + 0.5) * d;
}
__device__ __forceinline__ double departure(double c, double dt, double h) {
#pragma clang fp contract(off)
  return (c * dt) / h;
}

template <typename T>
__device__ __forceinline__ T vmin(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }

__device__ __forceinline__ float vfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double vfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// middle value of three numbers
__device__ __forceinline__ float med3(float a, float b, float c) {
  return __builtin_amdgcn_fmed3f(a, b, c);
}
__device__ __forceinline__ double med3(double a, double b, double c) {
  return vmax(vmin(a, b), vmin(vmax(a, b), c));
}
template <typename T>
__device__ __forceinline__ T min3(T a, T b, T c) { return vmin(vmin(a, b), c); }
template <typename T>
__device__ __forceinline__ T max3(T a, T b, T c) { return vmax(vmax(a, b), c); }

// minmod of two / four numbers through the median with zero: for equal
// signs the median of (a, b, 0) is the argument of smaller magnitude,
// otherwise it is zero.
template <typename T>
__device__ __forceinline__ T minmod2(T a, T b) { return med3(a, b, T(0)); }
template <typename T>
__device__ __forceinline__ T minmod4(T a, T b, T c, T d) {
  return med3(minmod2(a, b), minmod2(c, d), T(0));
}

template <typename T>
__device__ __forceinline__ T pp_theta(T u_up, T u) {
  T den = u_up - u;
  T t = den > T(0) ? u_up / den : T(0);
  return vmin(vmax(t, T(0)), T(1));
}

// Interface flux at the face between processing positions m and m+1
// (upwind cell m).  q holds r_{m-3}..r_{m+3} (seventh order) or
// r_{m-2}..r_{m+2} (fifth order).  d_m and DM_{m-1/2} come from the
// previous face; d_{m+1} and DM_{m+1/2} are returned for the next one.
template <typename T, int ORDER, int LIM>
__device__ __forceinline__ T face_flux(const T* q, const T* w, T z, T alpha, T& d_m, T& dm_prev) {
  constexpr int o = (ORDER == 7) ? 1 : 0;  // offset of the MP stencil in q
  T phi = w[0] * q[0];
#pragma unroll
  for (int k = 1; k < ORDER; ++k) phi = vfma(w[k], q[k], phi);
  if constexpr (LIM == SLMPP_LIM_NONE) {
    return phi;
  } else {
    const T fm1 = q[o + 1], f0 = q[o + 2], fp1 = q[o + 3], fp2 = q[o + 4];
    // App. A steps 4-7 (the early accept of step 3 is implied: a value
    // strictly between f_i and f* already lies in [f^min, f^max])
    const T d_new = vfma(T(-2), fp1, f0 + fp2);
    const T dm_new = minmod4(vfma(T(4), d_m, -d_new), vfma(T(4), d_new, -d_m),
                             d_m, d_new);
    const T slope = f0 - fm1;
    const T f_ul = vfma(alpha, slope, f0);
    const T f_md = vfma(T(-0.5), dm_new, T(0.5) * (f0 + fp1));
    const T f_lc = vfma(T(4.0 / 3.0), dm_prev, vfma(T(0.5), slope, f0));
    const T lo = vmax(min3(f0, fp1, f_md), min3(f0, f_ul, f_lc));
    const T hi = vmin(max3(f0, fp1, f_md), max3(f0, f_ul, f_lc));
    T phib = med3(phi, lo, hi);
    d_m = d_new;
    dm_prev = dm_new;
    if constexpr (LIM == SLMPP_LIM_MPP) {
      // PP limiter, Sec. 2.1.1: keep both half-updates non-negative
      const T tz = z + z;
      const T u_plus = vfma(-tz, phib, f0);
      const T u_minus = vfma(tz, phib, fp1);
      if (u_plus < T(0) || u_minus < T(0)) {
        T th = T(1);
        if (u_plus < T(0)) th = pp_theta(f0 - tz * f0, u_plus);
        if (u_minus < T(0)) th = vmin(th, pp_theta(vfma(tz, f0, fp1), u_minus));
        phib = th * phib + (T(1) - th) * f0;
      }
    }
    return phib;
  }
}

template <int MODE>
__device__ __forceinline__ int row_index(int r, int n, int G) {
  if constexpr (MODE == READ_DIRECT) {
    return r + G;
  } else if constexpr (MODE == READ_WRAP) {
    r %= n;
    if (r < 0) r += n;
    return r + G;
  } else {
    return min(max(r, -G), n + G - 1) + G;
  }
}

// Process positions [m0, m1) of one pencil whose input column starts at
// col (stride pitch) and whose output column starts at out.
template <typename T, int ORDER, int LIM, int MODE>
__device__ void sweep_segment(const T* __restrict__ col, T* __restrict__ out,
                              const ColParam<T>& cp, int n, int G, int pitch, int m0, int m1,
                              T alpha) {
  constexpr int H = (ORDER == 7) ? 3 : 2;  // window r_{m-H}..r_{m+H}
  constexpr int WIN = 2 * H + 1;
  T w[ORDER];
#pragma unroll
  for (int k = 0; k < ORDER; ++k) w[k] = cp.w[k];
  const T z = cp.z;
  const int dir = cp.dir;
  int r = cp.base + dir * (m0 - 1 - H);  // physical row of r_{m0-1-H}
  T q[WIN];
#pragma unroll
  for (int k = 0; k < WIN; ++k) {
    q[k] = col[row_index<MODE>(r, n, G) * pitch];
    r += dir;
  }
  // carried MP quantities for the face m0-1/2 (upwind cell m0-1):
  // d_{m0-1} and DM_{m0-3/2}
  constexpr int o = (ORDER == 7) ? 1 : 0;
  T d_prev = vfma(T(-2), q[o + 1], q[o] + q[o + 2]);     // d_{m0-2}
  T d_m = vfma(T(-2), q[o + 2], q[o + 1] + q[o + 3]);    // d_{m0-1}
  T dm_prev = minmod4(vfma(T(4), d_prev, -d_m), vfma(T(4), d_m, -d_prev),
                      d_prev, d_m);
  T f_left = face_flux<T, ORDER, LIM>(q, w, z, alpha, d_m, dm_prev);
  int orow = (dir > 0) ? m0 : (n - 1 - m0);
  for (int m = m0; m < m1; ++m) {
#pragma unroll
    for (int k = 0; k < WIN - 1; ++k) q[k] = q[k + 1];
    q[WIN - 1] = col[row_index<MODE>(r, n, G) * pitch];
    r += dir;
    const T f_right = face_flux<T, ORDER, LIM>(q, w, z, alpha, d_m, dm_prev);
    const T cell = q[H];  // r_m
    out[orow * pitch] = vfma(-z, f_right - f_left, cell);
    f_left = f_right;
    orow += dir;
  }
}

template <typename T, int ORDER>
__device__ void column_params(const SweepArgs& a, int64_t p, ColParam<T>& cp) {
  double c;
  if (a.cmode == SPEED_FROM_VELOCITY) {
    const int64_t j = p % a.inner;
    const int64_t jv = (j / a.vdiv) % a.nvl;
    c = cell_center(a.vlo, a.dv, jv);
  } else {
    c = a.accel[(p / a.inner) / a.xdiv];
  }
  const double xi = departure(c, a.dt, a.h);
  const int n = a.n;
  double zeta;
  int64_t N;
  if (!(fabs(xi) < 4.0e18)) {  // non-finite or absurd offset: poison the pencil
    N = 0;
    zeta = __builtin_nan("");
  } else {
    const double Nd = floor(xi + 0.5);
    zeta = xi - Nd;
    N = (int64_t)Nd;
  }
  if (a.bc == SLMPP_BC_PERIODIC) {
    N %= n;
    if (N < 0) N += n;
    if (N > n / 2) N -= n;
  } else {
    const int64_t lim = (int64_t)n + 64;
    N = N < -lim ? -lim : (N > lim ? lim : N);
  }
  const bool mirror = zeta < 0.0;
  const double az = mirror ? -zeta : zeta;
  cp.dir = mirror ? -1 : 1;
  cp.base = (int32_t)((mirror ? (int64_t)(n - 1) : 0) - N);
  const int64_t aN = N < 0 ? -N : N;
  cp.mode = aN <= a.nfast ? READ_DIRECT : (a.bc == SLMPP_BC_PERIODIC ? READ_WRAP : READ_CLAMP);
  cp.z = (T)az;
  cp.valid = 1;
#pragma unroll
  for (int k = 0; k < ORDER; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int j = ORDER - 1; j >= 0; --j) {
      Frac fr;
      if constexpr (ORDER == 7) {
        fr = kCsl7[k][j];
      } else {
        fr = kCsl5[k][j];
      }
      acc = acc * az + fr.num / fr.den;
    }
    cp.w[k] = (T)acc;
  }
}

template <typename T, int ORDER, int LIM>
__global__ void __launch_bounds__(256) sweep_tile_kernel(SweepArgs a, SweepPlan pl) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, W = pl.W, G = pl.G, pitch = pl.pitch;
  const int rows = n + 2 * G;
  T* tin = reinterpret_cast<T*>(smem);
  T* tout = tin + (size_t)rows * pitch;
  const size_t cp_off = ((size_t)(rows + n) * pitch * sizeof(T) + 15) & ~(size_t)15;
  ColParam<T>* cps = reinterpret_cast<ColParam<T>*>(smem + cp_off);
  T* f = reinterpret_cast<T*>(a.f);
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const T alpha = (T)a.alpha;
  const bool contiguous = (a.inner == 1);

  for (int64_t tile = blockIdx.x; tile < pl.tiles; tile += gridDim.x) {
    const int64_t p0 = tile * W;
    const int wv = (int)((a.npen - p0) < W ? (a.npen - p0) : W);  // valid pencils
    // ---- stream the tile in: global -> LDS rows [G, G+n) ----
    if (contiguous) {
      const int64_t gbase = p0 * n;
      const int total = wv * n;
      int jj = tid / n, i = tid - (tid / n) * n;
      const int sj = nthr / n, si = nthr - sj * n;
      for (int e = tid; e < total; e += nthr) {
        tin[(i + G) * pitch + jj] = f[gbase + e];
        i += si;
        jj += sj;
        if (i >= n) { i -= n; ++jj; }
      }
    } else {
      const int jj = tid % W;
      const int64_t p = p0 + jj;
      if (jj < wv) {
        const int64_t o = p / a.inner;
        const int64_t gb = o * (int64_t)n * a.inner + (p - o * a.inner);
        for (int i = tid / W; i < n; i += nthr / W) tin[(i + G) * pitch + jj] = f[gb + (int64_t)i * a.inner];
      }
    }
    // ---- ghost rows: periodic images or zeros ----
    for (int e = tid; e < 2 * G * W; e += nthr) {
      const int g = e / W, jj = e - g * W;
      const int gr = g < G ? g - G : n + (g - G);  // physical row of the ghost
      const int lrow = g < G ? g : n + g;          // LDS row
      T v = T(0);
      if (a.bc == SLMPP_BC_PERIODIC && jj < wv) {
        int src = gr % n;
        if (src < 0) src += n;
        const int64_t p = p0 + jj;
        const int64_t o = p / a.inner;
        v = f[o * (int64_t)n * a.inner + (int64_t)src * a.inner + (p - o * a.inner)];
      }
      tin[lrow * pitch + jj] = v;
    }
    // ---- per-pencil shift, direction and CSL weights ----
    for (int jj = tid; jj < W; jj += nthr) {
      if (jj < wv) {
        column_params<T, ORDER>(a, p0 + jj, cps[jj]);
      } else {
        ColParam<T> c{};
        c.dir = 1;
        c.mode = READ_DIRECT;
        c.valid = 0;
        cps[jj] = c;
      }
    }
    __syncthreads();
    // ---- compute: thread -> (pencil jj, segment s) ----
    {
      const int jj = tid % W;
      const int s = tid / W;
      const int S = nthr / W;
      const int R = (n + S - 1) / S;
      const int m0 = s * R;
      const int m1 = min(n, m0 + R);
      const ColParam<T> cp = cps[jj];
      if (cp.valid && m0 < m1) {
        const T* col = tin + jj;
        T* out = tout + jj;
        if (cp.mode == READ_DIRECT)
          sweep_segment<T, ORDER, LIM, READ_DIRECT>(col, out, cp, n, G, pitch, m0, m1, alpha);
        else if (cp.mode == READ_WRAP)
          sweep_segment<T, ORDER, LIM, READ_WRAP>(col, out, cp, n, G, pitch, m0, m1, alpha);
        else
          sweep_segment<T, ORDER, LIM, READ_CLAMP>(col, out, cp, n, G, pitch, m0, m1, alpha);
      }
    }
    __syncthreads();
    // ---- stream the tile out in place ----
    if (contiguous) {
      const int64_t gbase = p0 * n;
      const int total = wv * n;
      int jj = tid / n, i = tid - (tid / n) * n;
      const int sj = nthr / n, si = nthr - sj * n;
      for (int e = tid; e < total; e += nthr) {
        f[gbase + e] = tout[i * pitch + jj];
        i += si;
        jj += sj;
        if (i >= n) { i -= n; ++jj; }
      }
    } else {
      const int jj = tid % W;
      const int64_t p = p0 + jj;
      if (jj < wv) {
        const int64_t o = p / a.inner;
        const int64_t gb = o * (int64_t)n * a.inner + (p - o * a.inner);
        for (int i = tid / W; i < n; i += nthr / W) f[gb + (int64_t)i * a.inner] = tout[i * pitch + jj];
      }
    }
    __syncthreads();
  }
}

template <typename T, int ORDER, int LIM>
hipError_t launch_t(const SweepArgs& a, const SweepPlan& p, hipStream_t s) {
  if (p.tiles <= 0) return hipSuccess;
  auto kern = sweep_tile_kernel<T, ORDER, LIM>;
  if (p.lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  const int64_t grid = std::min<int64_t>(p.tiles, (int64_t)1 << 30);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(p.threads), p.lds_bytes, s, a, p);
  return hipGetLastError();
}

template <typename T, int ORDER>
hipError_t launch_o(int limiter, const SweepArgs& a, const SweepPlan& p, hipStream_t s) {
  switch (limiter) {
    case SLMPP_LIM_NONE: return launch_t<T, ORDER, SLMPP_LIM_NONE>(a, p, s);
    case SLMPP_LIM_MP: return launch_t<T, ORDER, SLMPP_LIM_MP>(a, p, s);
    default: return launch_t<T, ORDER, SLMPP_LIM_MPP>(a, p, s);
  }
}

size_t colparam_bytes(int dtype) {
  return dtype == SLMPP_F64 ? sizeof(ColParam<double>) : sizeof(ColParam<float>);
}

}  // namespace

SweepPlan plan_sweep(int dtype, int order, int32_t n, int64_t npen, int64_t inner, int32_t nfast,
                     int W_override, int S_override) {
  SweepPlan p{};
  const size_t es = dtype == SLMPP_F64 ? 8 : 4;
  const int gh = order == 7 ? 4 : 3;
  p.G = gh + nfast;
  const size_t budget = 80 * 1024;  // keeps two workgroups per CU at the largest tiles
  auto lds = [&](int W) {
    const size_t tiles = ((size_t)(2 * n + 2 * p.G) * (W + 1) * es + 15) & ~(size_t)15;
    return tiles + (size_t)W * colparam_bytes(dtype);
  };
  int W = 64;
  if (W_override > 0) {
    W = W_override;
  } else {
    while (W > 1 && lds(W) > budget) W /= 2;
  }
  (void)inner;
  int S;
  if (S_override > 0) {
    S = S_override;
  } else {
    S = std::max(1, 256 / W);
    S = std::min(S, std::max(1, n / 8));  // at least ~8 cells per segment
  }
  S = std::max(1, std::min(S, 256 / std::max(1, W)));
  p.W = W;
  p.S = S;
  p.threads = W * S;
  p.pitch = W + 1;
  p.lds_bytes = lds(W);
  p.tiles = (npen + W - 1) / W;
  return p;
}

hipError_t launch_sweep(int dtype, int order, int limiter, const SweepArgs& a, const SweepPlan& p,
                        hipStream_t s) {
  if (dtype == SLMPP_F64)
    return order == 7 ? launch_o<double, 7>(limiter, a, p, s) : launch_o<double, 5>(limiter, a, p, s);
  return order == 7 ? launch_o<float, 7>(limiter, a, p, s) : launch_o<float, 5>(limiter, a, p, s);
}

int32_t max_shift_velocity(double vlo, double dv, int32_t nvl, double dt, double h, int32_t n,
                           int32_t bc) {
  int64_t best = 0;
  for (int32_t j = 0; j < nvl; ++j) {
    double c, xi;
    {
#pragma clang fp contract(off)
      c = vlo + ((double)j + 0.5) * dv;
      xi = (c * dt) / h;
    }
    if (!(std::fabs(xi) < 4.0e18)) continue;
    int64_t N = (int64_t)std::floor(xi + 0.5);
    if (bc == SLMPP_BC_PERIODIC) {
      N %= n;
      if (N < 0) N += n;
      if (N > n / 2) N -= n;
    }
    const int64_t aN = N < 0 ? -N : N;
    best = std::max(best, aN);
  }
  return (int32_t)std::min<int64_t>(best, 64);
}

}  // namespace slmpp
