// Fused SL-MPP sweep kernels for gfx950.
//
// One launch advances every pencil along one axis of f by one
// semi-Lagrangian step (Sec. 2.1.2, Eq. (SL)):
//   xi = c dt / h  ->  integer shift N = floor(xi + 1/2), zeta = xi - N
//   Phi_{i-1/2}    =  CSL5 / CSL7 polynomial in zeta (rows C_j / D_j)
//   Phibar         =  MP constraint (App. A) on the 5-point stencil
//   Phihat         =  PP flux limiter (Sec. 2.1.1)
//   f_i^{n+1}      =  f_{i-N} - zeta (Phihat_{i+1/2} - Phihat_{i-1/2})
// For zeta < 0 the shifted pencil is processed in reverse order, the
// mirror image of the c > 0 construction the paper writes out.
//
// Two kernels per sweep:
//  * pencil_table_kernel: one entry per distinct speed (a velocity cell
//    centre for x-sweeps, a spatial cell for v-sweeps) holding the integer
//    shift, direction, |zeta| and the CSL flux as FIR weights w_k(|zeta|),
//    all computed in FP64 (rounded once to the storage type).
//  * sweep_kernel: a workgroup owns a tile of W whole pencils.  It streams
//    the tile from HBM into LDS once (16-byte vectors, coalesced along the
//    contiguous axis whichever way the pencils run), adds ghost rows
//    (periodic images or zeros), advances every pencil from LDS with a
//    register sliding window (each interface flux computed once and used
//    by both neighbouring cells; each thread owns a segment of R cells),
//    writes the results back into the LDS tile and streams it out in place.
//    A sweep therefore reads and writes f exactly once; halos stay on chip.
//    sweep_fast_kernel is its persistent form with the next tile prefetched
//    into registers (several runs of one geometry per launch for batched
//    ensembles); batch_sweep_kernel walks a list of tiles of many runs.
//  * kick_plane_kernel: the sweeps along the last two velocity axes of a
//    kick in one pass over f, whole velocity planes in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "slmpp_internal.hpp"

namespace slmpp {
namespace {

template <typename T>
struct alignas(16) PencilEntry {
  T w[7];        // FIR weights of the CSL flux at |zeta| (first ORDER used)
  T z;           // |zeta|
  T tz;          // 2 |zeta| (exact), the factor of the PP half-updates
  int32_t base;  // physical row read at processing position 0
  int16_t dir;   // +1 forward, -1 mirrored (zeta < 0)
  int16_t absN;  // |N| after periodic reduction (at most n + 64 <= 4160)
};
static_assert(sizeof(PencilEntry<float>) == 48 && sizeof(PencilEntry<double>) == 80,
              "pencil entries are 16-byte multiples");

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

// 2 |zeta| phib as one rounded product (never fused into a later add)
template <typename T>
__device__ __forceinline__ T pp_product(T tz, T phib) {
#pragma clang fp contract(off)
  return tz * phib;
}

template <typename T>
__device__ __noinline__ T pp_limit(T phib, T f0, T fp1, T tz, T p) {
  // theta = U^UP / (U^UP - U) on each side whose half-update is negative
  // (zero when the denominator is not positive), clamped to [0, 1]; the
  // flux moves toward the upwind value f0 by 1 - min(theta+, theta-).
  // p = 2 |zeta| phib (rounded); the half-updates and the limited flux are
  // formed without contraction, each operation rounded once.
#pragma clang fp contract(off)
  const T u_plus = f0 - p;
  const T u_minus = fp1 + p;
  T th = T(1);
  if (u_plus < T(0)) {
    const T up = f0 - tz * f0;
    const T den = up - u_plus;
    th = den > T(0) ? vmin(vmax(up / den, T(0)), T(1)) : T(0);
  }
  if (u_minus < T(0)) {
    const T up = fp1 + tz * f0;
    const T den = up - u_minus;
    th = vmin(th, den > T(0) ? vmin(vmax(up / den, T(0)), T(1)) : T(0));
  }
  return th * phib + (T(1) - th) * f0;
}

// App. A steps 4-7: the bounds f^min, f^max from the curvatures and the
// median of the flux with them.  The curvatures d_j = f_{j-1} + f_{j+1} -
// 2 f_j are formed as differences of the one-cell differences
// dll = f_{i-1} - f_{i-2}, dl = f_i - f_{i-1}, dr = f_{i+1} - f_i and
// drr = f_{i+2} - f_{i+1}, of which the face already holds dl and dr (and
// the previous face dll), so that nothing of these steps is computed
// outside the rare branch that needs them.
template <typename T>
__device__ __forceinline__ T mp_clamp(T phi, T dll, T dl, T dr, T drr, T f0, T fp1, T alpha) {
  const T dm1 = dl - dll;
  const T d0 = dr - dl;
  const T dp1 = drr - dr;
  const T dm4_plus = minmod4(vfma(T(4), d0, -dp1), vfma(T(4), dp1, -d0), d0, dp1);
  const T dm4_minus = minmod4(vfma(T(4), dm1, -d0), vfma(T(4), d0, -dm1), dm1, d0);
  const T f_ul = vfma(alpha, dl, f0);
  const T f_md = vfma(T(-0.5), dm4_plus, vfma(T(0.5), dr, f0));
  const T f_lc = vfma(T(4.0 / 3.0), dm4_minus, vfma(T(0.5), dl, f0));
  const T lo = vmax(min3(f0, fp1, f_md), min3(f0, f_ul, f_lc));
  const T hi = vmin(max3(f0, fp1, f_md), max3(f0, f_ul, f_lc));
  return med3(phi, lo, hi);
}

// Interface flux at the face between processing positions m and m+1
// (upwind cell m).  q holds r_{m-3}..r_{m+3} (seventh order) or
// r_{m-2}..r_{m+2} (fifth order); the MP constraint works on the five
// cells r_{m-2}..r_{m+2} in both cases.
template <typename T, int ORDER, int LIM>
__device__ __forceinline__ T face_flux(const T* q, const T* w, T tz, T alpha) {
  constexpr int o = (ORDER == 7) ? 1 : 0;  // offset of the MP stencil in q
  T phi = w[0] * q[0];
#pragma unroll
  for (int k = 1; k < ORDER; ++k) phi = vfma(w[k], q[k], phi);
  if constexpr (LIM == SLMPP_LIM_NONE) {
    return phi;
  } else {
    const T fm2 = q[o], fm1 = q[o + 1], f0 = q[o + 2], fp1 = q[o + 3], fp2 = q[o + 4];
    const T dl = f0 - fm1, dr = fp1 - f0;
    // App. A steps 2-3.  f* = f_i + minmod(f_{i+1} - f_i, alpha (f_i - f_{i-1}))
    // is the median of f_{i+1}, f^UL = f_i + alpha (f_i - f_{i-1}) and f_i
    // (adding f_i commutes with the median); it is formed that way, from
    // the same rounded f^UL that the bounds of step 6 use.  The flux is kept
    // when it lies between f_i and f*: f_i, f_{i+1} and f^UL each lie within
    // [f^min, f^max] (each bound is a min or max over sets holding f_i and
    // f_{i+1} or f_i and f^UL), so does every value between two of them, and
    // step 7 returns the flux unchanged there, in floating point as well.
    // The strict test of the text only sends the end points (a flux equal
    // to f_i, as in regions of zeros) through steps 4-7.
    const T fstar = med3(fp1, vfma(alpha, dl, f0), f0);
    const bool accept = med3(phi, f0, fstar) == phi;
    T phib = phi;
    // steps 4-7, skipped when every lane of the wavefront accepted (the
    // common case on smooth data)
    if (!__all(accept)) {
      // a zero the compiler cannot see through keeps the curvatures inside
      // this branch (it would otherwise form one per face for reuse by the
      // next face's branch: two instructions on every face)
      T zero = T(0);
      asm volatile("" : "+v"(zero));
      const T c = mp_clamp(phi, fm1 - fm2, dl + zero, dr + zero, fp2 - fp1, f0, fp1, alpha);
      phib = accept ? phi : c;
    }
    if constexpr (LIM == SLMPP_LIM_MPP) {
      // PP limiter, Sec. 2.1.1: keep both half-updates U+ = f_i - p and
      // U- = f_{i+1} + p (p = 2 |zeta| phib, rounded once) non-negative.
      // For floats a - b < 0 exactly when a < b, so the test needs only p.
      const T p = pp_product(tz, phib);
      if (p > f0 || -p > fp1) phib = pp_limit(phib, f0, fp1, tz, p);
    }
    return phib;
  }
}

enum : int32_t { READ_DIRECT = 0, READ_SAFE = 1 };

// Advance cells m0 .. m0+cnt-1 of one pencil (processing order).  `col`
// points at physical cell 0 of the pencil in the LDS tile; consecutive
// cells are `stride` elements apart and G ghost cells exist on both sides.
// READ_DIRECT assumes every read stays within the ghost cells; READ_SAFE
// wraps (periodic) or clamps onto the zero ghost cells (outflow).  With
// RC > 0 the segment length is RC and the results stay in out[]; with
// RC == 0 they are written to `ocol` (same geometry as col, no ghosts).
template <typename T, int ORDER, int LIM, int MODE, int RC>
__device__ __forceinline__ void advance(const T* __restrict__ col, int stride, int n, int G,
                                        int periodic, const PencilEntry<T>& e, int m0, int cnt,
                                        T alpha, T* out, T* __restrict__ ocol) {
  constexpr int H = (ORDER == 7) ? 3 : 2;  // window r_{m-H}..r_{m+H}
  constexpr int WIN = 2 * H + 1;
  T w[ORDER];
#pragma unroll
  for (int k = 0; k < ORDER; ++k) w[k] = e.w[k];
  const T z = e.z;
  const T tz = e.tz;
  const int dir = e.dir;
  int r = e.base + dir * (m0 - 1 - H);  // physical cell of r_{m0-1-H}
  const T* ptr = col + r * stride;      // READ_DIRECT walks a pointer
  const int step = dir * stride;
  auto fetch = [&]() -> T {
    T v;
    if constexpr (MODE == READ_DIRECT) {
      v = *ptr;
      ptr += step;
    } else {
      int rr = r;
      if (periodic) {
        rr %= n;
        if (rr < 0) rr += n;
      } else {
        rr = min(max(rr, -G), n + G - 1);  // ghost cells are zero
      }
      v = col[rr * stride];
      r += dir;
    }
    return v;
  };
  T q[WIN];
#pragma unroll
  for (int k = 0; k < WIN; ++k) q[k] = fetch();
  T f_left = face_flux<T, ORDER, LIM>(q, w, tz, alpha);
  if constexpr (RC > 0) {
#pragma unroll
    for (int k = 0; k < RC; ++k) {
#pragma unroll
      for (int j = 0; j < WIN - 1; ++j) q[j] = q[j + 1];
      q[WIN - 1] = fetch();
      const T f_right = face_flux<T, ORDER, LIM>(q, w, tz, alpha);
      out[k] = vfma(-z, f_right - f_left, q[H]);
      f_left = f_right;
    }
  } else {
    T* optr = ocol + ((dir > 0) ? m0 : (n - 1 - m0)) * stride;
    for (int k = 0; k < cnt; ++k) {
#pragma unroll
      for (int j = 0; j < WIN - 1; ++j) q[j] = q[j + 1];
      q[WIN - 1] = fetch();
      const T f_right = face_flux<T, ORDER, LIM>(q, w, tz, alpha);
      *optr = vfma(-z, f_right - f_left, q[H]);
      optr += step;
      f_left = f_right;
    }
  }
}

// advance() for READ_DIRECT with the stride and the processing direction
// known at compile time, so that the reads of a segment use fixed offsets
// from one address.  Same operations, same results.
template <typename T, int ORDER, int RC, int STRIDE, int DIR>
__device__ __forceinline__ void advance_ct(const T* __restrict__ col, const PencilEntry<T>& e,
                                           int m0, T alpha, T* out) {
  constexpr int H = (ORDER == 7) ? 3 : 2;
  constexpr int WIN = 2 * H + 1;
  constexpr int ST = DIR * STRIDE;
  T w[ORDER];
#pragma unroll
  for (int k = 0; k < ORDER; ++k) w[k] = e.w[k];
  const T z = e.z;
  const T tz = e.tz;
  const T* ptr = col + (e.base + DIR * (m0 - 1 - H)) * STRIDE;
  // the whole window of the segment is read before any flux is formed, so
  // that the LDS reads are in flight together (the branches of the MP and
  // PP steps would otherwise keep each read next to its first use)
  constexpr int NQ = RC + WIN;
  T q[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) q[k] = ptr[k * ST];
  T f_left = face_flux<T, ORDER, SLMPP_LIM_MPP>(q, w, tz, alpha);
#pragma unroll
  for (int k = 0; k < RC; ++k) {
    const T f_right = face_flux<T, ORDER, SLMPP_LIM_MPP>(q + k + 1, w, tz, alpha);
    out[k] = vfma(-z, f_right - f_left, q[k + 1 + H]);
    f_left = f_right;
  }
}

// Store the results of processing positions m0 .. m0 + RC - 1 of a pencil
// of n cells (physical cells m0 + k, or n - 1 - m0 - k when mirrored).
template <typename T, int RC, int STRIDE, int DIR>
__device__ __forceinline__ void store_ct(T* col, int n, int m0, const T* out) {
  T* op = col + ((DIR > 0) ? m0 : (n - 1 - m0)) * STRIDE;
#pragma unroll
  for (int k = 0; k < RC; ++k) op[k * DIR * STRIDE] = out[k];
}

// 16-byte vectors as native clang vector types (kept in registers)
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Vec;
template <>
struct Vec<float> {
  using type = vf4;
  static constexpr int N = 4;
};
template <>
struct Vec<double> {
  using type = vd2;
  static constexpr int N = 2;
};

// scatter / gather the components of a 16-byte vector to / from
// consecutive elements (component access keeps the vector in registers)
// sum of a vector's components in double (fused moment)
__device__ __forceinline__ double vsum(const vf4& v) {
  return ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
}
__device__ __forceinline__ double vsum(const vd2& v) { return v.x + v.y; }

__device__ __forceinline__ void put(float* d, const vf4& v) {
  d[0] = v.x;
  d[1] = v.y;
  d[2] = v.z;
  d[3] = v.w;
}
__device__ __forceinline__ void put(double* d, const vd2& v) {
  d[0] = v.x;
  d[1] = v.y;
}
__device__ __forceinline__ void get(const float* s, vf4& v) {
  v.x = s[0];
  v.y = s[1];
  v.z = s[2];
  v.w = s[3];
}
__device__ __forceinline__ void get(const double* s, vd2& v) {
  v.x = s[0];
  v.y = s[1];
}

// Result vector v of the elements at offset off from f: blended with
// fblend and stored to fout or f (see SweepArgs; STAGE false: plain store
// to f, for kernels that never run a TVD-RK stage); 16-byte aligned.
template <bool STAGE = true, typename T, typename V>
__device__ __forceinline__ void emit_vec(const SweepArgs& a, T* f, int64_t off, V v) {
  constexpr int VN = sizeof(V) / sizeof(T);
  if (!STAGE) {
    __builtin_nontemporal_store(v, reinterpret_cast<V*>(f + off));
    return;
  }
  if (a.fblend) {
    const T cb = (T)a.cb, cf = (T)a.cf;
    const V b = __builtin_nontemporal_load(
        reinterpret_cast<const V*>(reinterpret_cast<const T*>(a.fblend) + off));
#pragma unroll
    for (int c = 0; c < VN; ++c) v[c] = vfma(cb, b[c], cf * v[c]);
  }
  T* dst = a.fout ? reinterpret_cast<T*>(a.fout) : f;
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(dst + off));
}
// f as global memory: global (not flat) loads and stores of the fast
// kernel, whose address may then keep a wave-uniform base in scalar
// registers
template <typename V>
using GlobalPtr = __attribute__((address_space(1))) V*;
template <typename V>
__device__ __forceinline__ V global_load_nt(const V* p) {
  return __builtin_nontemporal_load((GlobalPtr<const V>)p);
}
template <typename V>
__device__ __forceinline__ void global_store_nt(V v, V* p) {
  __builtin_nontemporal_store(v, (GlobalPtr<V>)p);
}
// emit_vec for the vector `lane` of a row at the wave-uniform element
// offset uoff
template <typename T, typename V>
__device__ __forceinline__ void emit_vec_row(const SweepArgs& a, T* f, int64_t uoff, int lane, V v) {
  constexpr int VN = sizeof(V) / sizeof(T);
  if (a.fblend) {
    const T cb = (T)a.cb, cf = (T)a.cf;
    const V b = global_load_nt(reinterpret_cast<const V*>(reinterpret_cast<const T*>(a.fblend) + uoff) + lane);
#pragma unroll
    for (int c = 0; c < VN; ++c) v[c] = vfma(cb, b[c], cf * v[c]);
  }
  T* dst = a.fout ? reinterpret_cast<T*>(a.fout) : f;
  global_store_nt(v, reinterpret_cast<V*>(dst + uoff) + lane);
}
template <bool STAGE = true, typename T>
__device__ __forceinline__ void emit_one(const SweepArgs& a, T* f, int64_t off, T v) {
  if (!STAGE) {
    f[off] = v;
    return;
  }
  if (a.fblend) v = vfma((T)a.cb, reinterpret_cast<const T*>(a.fblend)[off], (T)a.cf * v);
  (a.fout ? reinterpret_cast<T*>(a.fout) : f)[off] = v;
}

// a / b for non-negative 64-bit values, in 32-bit arithmetic when both fit
__device__ __forceinline__ int64_t udiv(int64_t a, int64_t b) {
  if (((a | b) >> 31) == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
  return a / b;
}

// LDS tile layouts.  Strided axis: row-major [cell][pencil] with pitch W
// (a tile row is W consecutive elements of f; lanes of a wave read W
// different pencils of one row, so every bank is distinct).  Contiguous
// axis: pencil-major [pencil][cell] with an odd pitch (W pencils are W*n
// consecutive elements of f; lanes reading cell r of W pencils hit
// distinct banks).  Both layouts carry G ghost cells before and after each
// pencil.
// RC: cells per thread (0: runtime segment length).  WT: pencils per tile
// as a compile-time constant (0: runtime), which turns the thread -> (pencil,
// segment) and vector -> (row, column) maps into shifts and multiplies.
template <typename T, int ORDER, int LIM, int RC, int WT, bool STAGE = true>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, const SweepPlan& pl,
                                           const PencilEntry<T>* __restrict__ table,
                                           int64_t tile_index, unsigned char* smem) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::N;
  const int n = a.n, G = pl.G, P = pl.pitch;
  const int W = WT > 0 ? WT : pl.W;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const bool periodic = a.bc == SLMPP_BC_PERIODIC;
  const bool contiguous = a.inner == 1;
  // element offset of ghost-extended cell g (0 <= g < n+2G) of pencil jj
  // in the tile: contiguous jj*P + g, strided g*W + jj
  const int cstride = contiguous ? 1 : W;  // between cells of a pencil
  const int pstride = contiguous ? P : 1;  // between pencils
  const int tile_elems = contiguous ? W * P : (n + 2 * G) * W;
  T* tile = reinterpret_cast<T*>(smem);
  const size_t tile_bytes = ((size_t)tile_elems * sizeof(T) + 15) & ~(size_t)15;
  PencilEntry<T>* ent = reinterpret_cast<PencilEntry<T>*>(smem + tile_bytes);
  T* tout = reinterpret_cast<T*>(ent + W);  // RC == 0 only: tile_elems
  T* f = reinterpret_cast<T*>(a.f);
  const T alpha = (T)a.alpha;

  const int64_t p0 = tile_index * W;
  const int wv = (int)min<int64_t>(W, a.npen - p0);
  const bool block = !contiguous && (a.inner % W == 0);
  int64_t gbase = 0, o0 = 0, j0 = 0;
  if (contiguous) {
    gbase = p0 * n;
  } else if (block) {
    o0 = udiv(p0, a.inner);
    j0 = p0 - o0 * a.inner;
    gbase = o0 * (int64_t)n * a.inner + j0;
  }

  // ---- per-pencil table entry ------------------------------------------
  int need_safe = 0;
  for (int jj = tid; jj < W; jj += nthr) {
    if (jj < wv) {
      const int64_t p = p0 + jj;
      int64_t o, j;
      if (contiguous) {
        o = p;
        j = 0;
      } else if (block) {
        o = o0;
        j = j0 + jj;
      } else {
        o = udiv(p, a.inner);
        j = p - o * a.inner;
      }
      const int64_t idx = a.cmode == SPEED_FROM_VELOCITY ? udiv(j, a.vdiv) % a.nvl : udiv(o, a.xdiv);
      const PencilEntry<T>* src = table + idx;
      ent[jj] = *src;
      need_safe |= src->absN > a.nfast;
    } else {
      ent[jj].z = T(0);
      ent[jj].tz = T(0);
      ent[jj].base = 0;
      ent[jj].dir = 1;
      ent[jj].absN = 0;
    }
  }

  // ---- stream the tile in: global -> LDS ------------------------------------
  // Loads are issued in batches of KB vectors per thread before any of them
  // is written to LDS, so each thread keeps KB requests in flight.  Whole
  // vectors of f are loaded and stored nontemporally (read and written once).
  constexpr int KB = 6;
  const bool vec_strided = block && (W % VN) == 0 && (a.inner % VN) == 0 && (gbase % VN) == 0 &&
                           (nthr % (W / VN)) == 0;
  // strided periodic tiles with G <= n fill their ghost rows while staging
  // (the generic strided path needs every pencil column loaded: nthr % W == 0)
  const bool wrap_rows = !contiguous && periodic && G <= n && (vec_strided || (nthr % W) == 0);
  if (contiguous) {
    const int total = wv * n;
    if ((n % VN) == 0) {
      // vector e4 holds cells i..i+VN-1 of pencil jj (n % VN == 0: never split)
      const int nvec = total / VN;
      const int stepE = nthr * VN;
      const int dj = stepE / n, di = stepE - dj * n;
      int jj = (tid * VN) / n, i = tid * VN - jj * n;
      const V* src = reinterpret_cast<const V*>(f + gbase);
      for (int b0 = tid; b0 < nvec; b0 += KB * nthr) {
        V buf[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k)
          if (b0 + k * nthr < nvec) buf[k] = __builtin_nontemporal_load(src + b0 + k * nthr);
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (b0 + k * nthr < nvec) {
            put(tile + jj * P + G + i, buf[k]);
            i += di;
            jj += dj;
            if (i >= n) {
              i -= n;
              ++jj;
            }
          }
        }
      }
    } else {
      for (int e2 = tid; e2 < total; e2 += nthr) {
        const int jj = e2 / n, i = e2 - jj * n;
        tile[jj * P + G + i] = f[gbase + e2];
      }
    }
  } else if (vec_strided) {
    const int cpr = W / VN;  // vectors per row; nthr % cpr == 0
    const int c = tid % cpr;
    const int di = nthr / cpr;
    const int i0 = tid / cpr;
    const T* gp = f + gbase + (int64_t)i0 * a.inner + c * VN;
    const int64_t gstep = (int64_t)di * a.inner;
    for (int ib = i0; ib < n; ib += KB * di, gp += KB * gstep) {
      V buf[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (ib + k * di < n)
          buf[k] = __builtin_nontemporal_load(reinterpret_cast<const V*>(gp + k * gstep));
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (ib + k * di < n) {
          const int i = ib + k * di;
          V* dst = reinterpret_cast<V*>(tile + (i + G) * W + c * VN);
          *dst = buf[k];
          if (wrap_rows) {
            if (i < G) *reinterpret_cast<V*>(tile + (i + G + n) * W + c * VN) = buf[k];
            if (i >= n - G) *reinterpret_cast<V*>(tile + (i + G - n) * W + c * VN) = buf[k];
          }
        }
      }
    }
  } else {
    // generic strided tile: thread -> fixed pencil column, rows stepped
    const int jj = tid % W;
    if (jj < wv && (nthr % W) == 0) {
      const int64_t p = p0 + jj;
      const int64_t o = udiv(p, a.inner);
      const T* gp = f + o * (int64_t)n * a.inner + (p - o * a.inner);
      const int di = nthr / W;
      for (int ib = tid / W; ib < n; ib += KB * di) {
        T buf[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k)
          if (ib + k * di < n) buf[k] = gp[(int64_t)(ib + k * di) * a.inner];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (ib + k * di < n) {
            const int i = ib + k * di;
            tile[(i + G) * W + jj] = buf[k];
            if (wrap_rows) {
              if (i < G) tile[(i + G + n) * W + jj] = buf[k];
              if (i >= n - G) tile[(i + G - n) * W + jj] = buf[k];
            }
          }
        }
      }
    }
  }
  // zero ghost cells (outflow); periodic images are copied after the barrier
  if (!periodic) {
    for (int e2 = tid; e2 < 2 * G * W; e2 += nthr) {
      const int g = e2 / W, jj = e2 - g * W;
      tile[jj * pstride + (g < G ? g : n + g) * cstride] = T(0);
    }
  }
  const bool safe = __syncthreads_or(need_safe) != 0;
  if (periodic && G > 0 && !wrap_rows) {
    for (int e2 = tid; e2 < 2 * G * W; e2 += nthr) {
      const int g = e2 / W, jj = e2 - g * W;
      const int pr = g < G ? g - G : n + (g - G);  // physical cell of the ghost
      int sp = pr < 0 ? pr + n : (pr >= n ? pr - n : pr);
      if (G > n) {  // pencils shorter than the ghost width
        sp = pr % n;
        if (sp < 0) sp += n;
      }
      tile[jj * pstride + (g < G ? g : n + g) * cstride] = tile[jj * pstride + (sp + G) * cstride];
    }
    __syncthreads();
  }

  // ---- compute: thread -> (pencil jj, segment s) -------------------------
  const int jj = tid % W;
  const int s = tid / W;
  const PencilEntry<T> e = ent[jj];
  const T* col = tile + jj * pstride + G * cstride;  // physical cell 0
  if constexpr (RC > 0) {
    T out[RC > 0 ? RC : 1];
    const int m0 = s * RC;
    const bool act = jj < wv && m0 < n;
    if (act) {
      if (!safe)
        advance<T, ORDER, LIM, READ_DIRECT, RC>(col, cstride, n, G, periodic, e, m0, RC, alpha,
                                                out, nullptr);
      else
        advance<T, ORDER, LIM, READ_SAFE, RC>(col, cstride, n, G, periodic, e, m0, RC, alpha, out,
                                              nullptr);
    }
    __syncthreads();
    if (act) {
      T* op = tile + jj * pstride + (G + ((e.dir > 0) ? m0 : (n - 1 - m0))) * cstride;
      const int ostep = e.dir * cstride;
#pragma unroll
      for (int k = 0; k < RC; ++k) {
        *op = out[k];
        op += ostep;
      }
    }
  } else {
    const int S = nthr / W;
    const int R = (n + S - 1) / S;
    const int m0 = s * R;
    const int cnt = min(n, m0 + R) - m0;
    if (jj < wv && cnt > 0) {
      T* ocol = tout + jj * pstride + G * cstride;
      if (!safe)
        advance<T, ORDER, LIM, READ_DIRECT, 0>(col, cstride, n, G, periodic, e, m0, cnt, alpha,
                                               nullptr, ocol);
      else
        advance<T, ORDER, LIM, READ_SAFE, 0>(col, cstride, n, G, periodic, e, m0, cnt, alpha,
                                             nullptr, ocol);
    }
  }
  __syncthreads();
  const T* res = RC > 0 ? tile : tout;  // same geometry as the tile

  // ---- fused velocity moment (batched 1D1V x_1 sweeps: the pencils of a
  // tile are consecutive velocity cells): each lane adds 8 consecutive
  // results of a tile row in double and stores that chunk sum at
  // mom[(p0 / 8 + chunk) n + i]; chunks of 8 for every tile width, so the
  // moment does not depend on W (W and the number of velocity cells are
  // multiples of 8 here, hence so is wv)
  if (!contiguous && a.mom != nullptr) {
    const int CPR = W / 8;
    const int q = tid % CPR;
    if (8 * q < wv) {
      for (int i = tid / CPR; i < n; i += nthr / CPR) {
        const T* row = res + (i + G) * W + 8 * q;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) v += (double)row[k];
        a.mom[(p0 / 8 + q) * n + i] = v;
      }
    }
  }

  // ---- stream the tile out in place ---------------------------------------
  if (contiguous) {
    const int total = wv * n;
    if ((n % VN) == 0) {
      const int nvec = total / VN;
      const int stepE = nthr * VN;
      const int dj = stepE / n, di = stepE - dj * n;
      int c = (tid * VN) / n, i = tid * VN - c * n;
      for (int b0 = tid; b0 < nvec; b0 += KB * nthr) {
        V buf[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (b0 + k * nthr < nvec) {
            get(res + c * P + G + i, buf[k]);
            i += di;
            c += dj;
            if (i >= n) {
              i -= n;
              ++c;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
          if (b0 + k * nthr < nvec) emit_vec<STAGE>(a, f, gbase + (int64_t)(b0 + k * nthr) * VN, buf[k]);
      }
    } else {
      for (int e2 = tid; e2 < total; e2 += nthr) {
        const int c = e2 / n, i = e2 - c * n;
        emit_one<STAGE>(a, f, gbase + e2, res[c * P + G + i]);
      }
    }
  } else if (vec_strided) {
    const int cpr = W / VN;
    const int c = tid % cpr;
    const int di = nthr / cpr;
    const int i0 = tid / cpr;
    int64_t go = gbase + (int64_t)i0 * a.inner + c * VN;
    const int64_t gstep = (int64_t)di * a.inner;
    for (int ib = i0; ib < n; ib += KB * di, go += KB * gstep) {
      V buf[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (ib + k * di < n) buf[k] = *reinterpret_cast<const V*>(res + (ib + k * di + G) * W + c * VN);
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (ib + k * di < n) emit_vec<STAGE>(a, f, go + k * gstep, buf[k]);
    }
  } else {
    const int c = tid % W;
    if (c < wv && (nthr % W) == 0) {
      const int64_t p = p0 + c;
      const int64_t o = udiv(p, a.inner);
      const int64_t go = o * (int64_t)n * a.inner + (p - o * a.inner);
      for (int i = tid / W; i < n; i += nthr / W)
        emit_one<STAGE>(a, f, go + (int64_t)i * a.inner, res[(i + G) * W + c]);
    }
  }
}

template <typename T, int ORDER, int LIM, int RC, int WT>
__global__ void __launch_bounds__(256) sweep_kernel(SweepArgs a, SweepPlan pl,
                                                    const PencilEntry<T>* __restrict__ table) {
  extern __shared__ __align__(16) unsigned char smem[];
  sweep_tile<T, ORDER, LIM, RC, WT>(a, pl, table, (int64_t)blockIdx.x, smem);
}

// Fast path: persistent workgroups over whole tiles with software prefetch.
// f is streamed with nontemporal loads and stores (each element is read and
// written once per sweep; measured 4-5% faster than cached accesses).
// Each thread owns RC cells of one pencil and, for the data movement, RC
// elements of the tile (RC/VN vectors at fixed offsets, the same for every
// tile), so the loads of the next tile can be issued into registers before
// the current tile is computed.  Requirements checked on the host: SL-MPP,
// W divides `inner` (strided) or inner == 1 (contiguous), RC divides n,
// VN divides RC (and n when contiguous), and all pencil / cell counts of a
// block fit in 32 bits.
// Strided 256-pencil tiles (48-cell FP32 pencils) run 512 threads in two
// segments with at most 128 VGPRs, so that two workgroups share a CU: the
// register bound costs a few spilled values per tile, and the wider rows
// (1 KiB per row and tile) and the loads of two tiles in flight per CU
// make these sweeps 4-14% faster than 128-pencil tiles at 48^3 x 48^3.
template <typename T, int ORDER, int RC, int WT, bool CONTIG, bool MOM>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, WT == 256 ? 512 : 256),
                               amdgpu_waves_per_eu(WT == 256 ? 4 : 1)))
sweep_fast_kernel(SweepArgs a, SweepPlan pl,
                                                         const PencilEntry<T>* __restrict__ table) {
  extern __shared__ __align__(16) unsigned char smem[];
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::N;
  constexpr int NV = RC / VN;  // vectors per thread and tile
  constexpr int W = WT;
  static_assert(RC % VN == 0, "segment length must be a multiple of the vector width");
  const int n = a.n, G = pl.G, P = pl.pitch;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int S = WT == 256 ? 2 : nthr / W;
  const bool periodic = a.bc == SLMPP_BC_PERIODIC;
  const int cstride = CONTIG ? 1 : W;
  const int pstride = CONTIG ? P : 1;
  const int tile_elems = CONTIG ? W * P : (n + 2 * G) * W;
  T* tile = reinterpret_cast<T*>(smem);
  const size_t tile_bytes = ((size_t)tile_elems * sizeof(T) + 15) & ~(size_t)15;
  PencilEntry<T>* ent = reinterpret_cast<PencilEntry<T>*>(smem + tile_bytes);
  T* f = reinterpret_cast<T*>(a.f);
  const T alpha = (T)a.alpha;
  const uint32_t inner = (uint32_t)a.inner;

  // per-thread element map of the data movement (identical for every tile)
  int loff[NV];       // LDS element offset of vector k
  int64_t goff0;      // global element offset of vector 0 relative to the tile
  int64_t gstep;      // between consecutive vectors of the thread
  // strided 256-pencil tiles: a row of the tile is the 64 vectors of one
  // wavefront, so the row part of each address is wave-uniform
  constexpr bool ROWWAVE = !CONTIG && W / VN == 64;
  int64_t urow = 0;   // wave-uniform row offset of vector 0
  int vlane = 0;      // vector of the lane within its row
  int vlim[NV];       // vector k exists when the tile has more than vlim[k] valid pencils
  if constexpr (CONTIG) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = VN * (tid + k * nthr);
      const int pj = e / n;
      loff[k] = pj * P + G + (e - pj * n);
      vlim[k] = pj;
    }
    goff0 = (int64_t)VN * tid;
    gstep = (int64_t)VN * nthr;
  } else {
    constexpr int cpr = W / VN;
    const int c = tid % cpr, i0 = tid / cpr;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      loff[k] = (i0 + k * S * VN + G) * W + c * VN;
      vlim[k] = c * VN;
    }
    goff0 = (int64_t)i0 * inner + c * VN;
    gstep = (int64_t)S * VN * inner;
    if constexpr (ROWWAVE) {
      urow = (int64_t)__builtin_amdgcn_readfirstlane(i0) * inner;
      vlane = c;
    }
  }
  // strided periodic tiles with G <= n fill their ghost rows while staging
  const bool wrap_rows = !CONTIG && periodic && G <= n;
  int i0s = 0;  // first physical row of this thread's vectors (strided)
  if constexpr (!CONTIG) i0s = tid / (W / VN);
  // zero ghost cells once: interior writes never touch them
  if (!periodic) {
    for (int e2 = tid; e2 < 2 * G * W; e2 += nthr) {
      const int g = e2 / W, c = e2 - g * W;
      tile[c * pstride + (g < G ? g : n + g) * cstride] = T(0);
    }
  }
  const int jj = tid % W;
  const int s = tid / W;
  const int m0 = s * RC;

  auto tile_base = [&](int64_t t, int& wv) -> int64_t {
    const int64_t p0 = t * W;
    wv = (int)min<int64_t>(W, a.npen - p0);
    if constexpr (CONTIG) {
      return p0 * n;
    } else {
      const uint32_t o0 = (uint32_t)p0 / inner;
      const uint32_t j0 = (uint32_t)p0 - o0 * inner;
      return (int64_t)o0 * n * inner + j0;
    }
  };

  // run and local tile of global tile tt (several runs: see SweepArgs)
  auto locate = [&](int64_t tt, int64_t& lt) -> int {
    if (a.fmulti == nullptr) {
      lt = tt;
      return 0;
    }
    const int r = (int)(tt / a.tpr);
    lt = tt - (int64_t)r * a.tpr;
    return r;
  };

  auto load_vec = [&](const T* fb, int64_t gb, int k) -> V {
    if constexpr (ROWWAVE)
      return global_load_nt(reinterpret_cast<const V*>(fb + (gb + urow + k * gstep)) + vlane);
    else
      return global_load_nt(reinterpret_cast<const V*>(fb + gb + goff0 + k * gstep));
  };

  V pf[NV];
  int64_t t = blockIdx.x;
  int wv_next = 0;
  int64_t gb_next = 0, lt_next = 0;
  int r_next = 0;
  T* f_next = f;
  if (t < pl.tiles) {
    r_next = locate(t, lt_next);
    if (a.fmulti) f_next = reinterpret_cast<T*>(a.fmulti[r_next]);
    gb_next = tile_base(lt_next, wv_next);
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (vlim[k] < wv_next)
        pf[k] = load_vec(f_next, gb_next, k);
  }
  for (; t < pl.tiles; t += gridDim.x) {
    const int wv = wv_next;
    const int64_t gbase = gb_next;
    const int64_t p0 = lt_next * W;
    T* const fc = f_next;
    const PencilEntry<T>* tabc =
        a.fmulti ? reinterpret_cast<const PencilEntry<T>*>(a.tmulti[r_next]) : table;
    // ---- pencil entries of this tile ----
    int need_safe = 0;
    if (tid < W) {
      if (tid < wv) {
        uint32_t idx;
        if constexpr (CONTIG) {
          const uint32_t o = (uint32_t)(p0 + tid);
          idx = a.cmode == SPEED_FROM_VELOCITY ? 0u : o / (uint32_t)a.xdiv;
        } else {
          const uint32_t o0 = (uint32_t)p0 / inner;
          const uint32_t j = (uint32_t)p0 - o0 * inner + tid;
          idx = a.cmode == SPEED_FROM_VELOCITY ? (j / (uint32_t)a.vdiv) % (uint32_t)a.nvl
                                               : o0 / (uint32_t)a.xdiv;
        }
        const PencilEntry<T>* src = tabc + idx;
        ent[tid] = *src;
        need_safe = src->absN > a.nfast;
      } else {
        ent[tid].z = T(0);
        ent[tid].tz = T(0);
        ent[tid].base = 0;
        ent[tid].dir = 1;
        ent[tid].absN = 0;
      }
    }
    // ---- prefetched data -> LDS ----
    // (strided periodic tiles also write the first and last G rows into the
    // ghost rows on the other side, which saves a copy pass and a barrier)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if (vlim[k] < wv) {
        put(tile + loff[k], pf[k]);
        if constexpr (!CONTIG) {
          if (wrap_rows) {
            const int i = i0s + k * S * VN;  // physical row of vector k
            if (i < G) put(tile + loff[k] + n * W, pf[k]);
            if (i >= n - G) put(tile + loff[k] - n * W, pf[k]);
          }
        }
      }
    }
    const bool safe = __syncthreads_or(need_safe) != 0;
    if (periodic && !wrap_rows) {
      for (int e2 = tid; e2 < 2 * G * W; e2 += nthr) {
        const int g = e2 / W, c = e2 - g * W;
        const int pr = g < G ? g - G : n + (g - G);
        int sp = pr < 0 ? pr + n : (pr >= n ? pr - n : pr);
        if (G > n) {
          sp = pr % n;
          if (sp < 0) sp += n;
        }
        tile[c * pstride + (g < G ? g : n + g) * cstride] = tile[c * pstride + (sp + G) * cstride];
      }
      __syncthreads();
    }
    // ---- issue the loads of the next tile ----
    if (t + gridDim.x < pl.tiles) {
      r_next = locate(t + gridDim.x, lt_next);
      if (a.fmulti) f_next = reinterpret_cast<T*>(a.fmulti[r_next]);
      gb_next = tile_base(lt_next, wv_next);
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (vlim[k] < wv_next)
          pf[k] = load_vec(f_next, gb_next, k);
    }
    // ---- compute ----
    const PencilEntry<T> e = ent[jj];
    const bool act = jj < wv;
    T out[RC];
    const T* col = tile + jj * pstride + G * cstride;
    if (act) {
      if (!safe)
        advance<T, ORDER, SLMPP_LIM_MPP, READ_DIRECT, RC>(col, cstride, n, G, periodic, e, m0, RC,
                                                          alpha, out, nullptr);
      else
        advance<T, ORDER, SLMPP_LIM_MPP, READ_SAFE, RC>(col, cstride, n, G, periodic, e, m0, RC,
                                                        alpha, out, nullptr);
    }
    __syncthreads();
    if (act) {
      T* op = tile + jj * pstride + (G + ((e.dir > 0) ? m0 : (n - 1 - m0))) * cstride;
      const int ostep = e.dir * cstride;
#pragma unroll
      for (int k = 0; k < RC; ++k) {
        *op = out[k];
        op += ostep;
      }
    }
    __syncthreads();
    // ---- stream the results out ----
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if (vlim[k] < wv) {
        V v;
        get(tile + loff[k], v);
        if constexpr (ROWWAVE)
          emit_vec_row(a, fc, gbase + urow + k * gstep, vlane, v);
        else
          emit_vec(a, fc, gbase + goff0 + k * gstep, v);
      }
    }
    if constexpr (MOM) {
      // fused velocity moment (strided tiles of 64, 128 or 256 pencils within
      // one velocity block): LPR lanes per tile row each add 16 of the
      // row's pencils in double (16-byte reads, start rotated by the row so
      // the lanes of a wavefront spread over the LDS banks), then the
      // partial sums are combined in a fixed order and stored per tile and
      // row
      static_assert(!CONTIG && (WT == 64 || WT == 128 || WT == 256), "fused moment needs wide strided tiles");
      constexpr int LPR = WT / 16;
      const int q = tid % LPR;
      for (int i = tid / LPR; i < n; i += nthr / LPR) {
        const T* row = tile + (i + G) * W;
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < 16 / VN; ++r) {
          V x;
          get(row + ((q * 16 + r * VN + 4 * i) & (WT - 1)), x);
          v += vsum(x);
        }
#pragma unroll
        for (int off = 1; off < LPR; off <<= 1) v += __shfl_xor(v, off, LPR);
        if (q == 0) a.mom[t * n + i] = v;
      }
    }
    // the row sums read every thread's vectors: the next tile's LDS writes
    // wait for them.  Without them no barrier is needed here: the next
    // tile first writes this thread's own data-movement vectors (at the
    // offsets it has just read), ghost rows and pencil entries, none of
    // which another thread reads before the next barrier.
    if constexpr (MOM) __syncthreads();
  }
}

// The last two velocity axes of a kick in one pass.  The acceleration
// depends on x only, so all pencils along v_{D-1} of a plane
// (x, v_1..v_{D-2}) share one shift and one set of weights, and so do all
// pencils along v_D; and a plane of N x N cells is one contiguous block of
// f.  A workgroup stages PB planes at a time in LDS, each inside a ring of
// G zero cells (outflow), advances the v_{D-1} pencils, writes the results
// back into the plane, advances the v_D pencils of the updated plane and
// streams the planes out: the two sweeps one after the other, cell for
// cell, for one read and one write of f.  Persistent over tiles of PB
// consecutive planes; the next tile's data are loaded into registers
// before the current tile is computed (as in sweep_fast_kernel).
//
// Threads are segment-major: thread t advances cells s R .. s R + R - 1 of
// pencil u = t mod (PB N) (plane u / N, pencil u mod N) with s = t / (PB N),
// so that where PB N is 64 (32^2 planes in pairs, 64^2 planes) every
// wavefront holds one segment and the wave-uniform skip of the MP bounds
// (App. A steps 4-7) is lost only in the wavefronts whose segment contains
// a rejecting face.  With UNI the PB planes of a tile belong to one spatial
// cell (vouter a multiple of PB): the two pencil entries are uniform over
// the workgroup and live in scalar registers.  (Four 48^2 planes per
// workgroup with one segment per wavefront were measured slower than one
// plane per workgroup: 33-38 ms against 25 ms per pass at 48^3 x 48^3, for
// want of wavefronts per CU.)
constexpr int kPlaneFast = 4;  // integer shifts read directly in the plane kernel

template <typename T, int ORDER, int N>
struct PlaneShape {
  // cells per thread (FP32 64^2 planes: 512 threads of 8 cells, whose extra
  // waves outweigh the segment-boundary faces they add)
  static constexpr int R = N == 64 ? (sizeof(T) == 4 ? 8 : 16) : (N == 48 ? 12 : 8);
  static constexpr int S = N / R;                               // segments per pencil
  static constexpr int PB = sizeof(T) == 4 ? (N == 24 ? 3 : N == 32 ? 2 : 1) : (N == 24 ? 2 : 1);
  static constexpr int threads = PB * N * S;
  // ring width (shifts up to kPlaneFast cells read the ring directly)
  static constexpr int G = (ORDER == 7 ? 4 : 3) + kPlaneFast;
  // odd row pitch: the rows of one plane start on distinct banks
  static constexpr int P = (N + 2 * G) | 1;
  // plane stride: the plane's rows padded to N (mod 64) elements, so that
  // with PB N = 64 the two planes of a wavefront fall on disjoint banks
  static constexpr int rows = (N + 2 * G) * P;
  static constexpr int PS = PB == 1 ? rows : rows + (((N - rows) % 64) + 64) % 64;
};

// A pencil entry read through the constant address space: the tables are
// not written while a sweep runs, so where the address is uniform over the
// wavefront the compiler loads the entry with scalar loads and keeps it in
// scalar registers (its weights then enter the FMAs as scalar operands).
template <typename T>
__device__ __forceinline__ PencilEntry<T> load_entry_uniform(const PencilEntry<T>* p) {
  constexpr int NW = sizeof(PencilEntry<T>) / 4;
  using CW = const __attribute__((address_space(4))) uint32_t*;
  const CW q = (CW)(p);
  uint32_t w[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) w[i] = q[i];
  PencilEntry<T> e;
  __builtin_memcpy(&e, w, sizeof(e));
  return e;
}
template <typename P>
__device__ __forceinline__ P load_ptr_uniform(const P* p) {
  using CU = const __attribute__((address_space(4))) uint64_t*;
  return reinterpret_cast<P>(static_cast<uintptr_t>(*(CU)(p)));
}

template <typename T, int ORDER, int N, bool UNI>
__global__ void __launch_bounds__((PlaneShape<T, ORDER, N>::threads))
    kick_plane_kernel(SweepArgs a, PlanePlan pl, const PencilEntry<T>* __restrict__ tabA,
                      const PencilEntry<T>* __restrict__ tabB) {
  extern __shared__ __align__(16) unsigned char smem[];
  using V = typename Vec<T>::type;
  using Sh = PlaneShape<T, ORDER, N>;
  constexpr int VN = Vec<T>::N;
  constexpr int R = Sh::R, S = Sh::S, PB = Sh::PB, NT = Sh::threads;
  constexpr int G = Sh::G, P = Sh::P, PS = Sh::PS;
  constexpr int NN = N * N;
  constexpr int PN = PB * N;                // pencils of one segment row of the tile
  constexpr int NVEC = PB * NN / VN;       // 16-byte vectors per tile
  constexpr int NV = (NVEC + NT - 1) / NT;  // per thread
  static_assert(N % VN == 0 && N % R == 0 && PB >= 1 && NT <= 1024, "plane shape");
  const int tid = threadIdx.x;
  T* lds = reinterpret_cast<T*>(smem);
  T* f = reinterpret_cast<T*>(a.f);
  const T alpha = (T)a.alpha;
  // zero the planes with their rings once (interior writes never touch the
  // rings); the barrier orders these stores before the first tile's data
  for (int e = tid; e < PB * PS; e += NT) lds[e] = T(0);
  __syncthreads();
  // data movement map: vector k of this thread is tile vector tid + NT k,
  // in plane vq[k] (PB: none) at LDS offset loff[k]
  int loff[NV], vq[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int v = tid + NT * k;
    if (v < NVEC) {
      const int e = v * VN;
      const int q = e / NN, rem = e - q * NN;
      const int ia = rem / N, ib = rem - ia * N;
      loff[k] = q * PS + (ia + G) * P + G + ib;
      vq[k] = q;
    } else {
      loff[k] = 0;
      vq[k] = PB;
    }
  }
  // compute map (segment-major): plane cq, pencil cj, cells m0 .. m0 + R - 1
  // of segment s.  With four segments and a wavefront holding parts of two,
  // the segments are laid out in the order 2, 0, 3, 1 (wavefronts hold
  // segments 2 and 0, 0 and 3, 3 and 1), so that a wavefront's lanes fail
  // the early MP accept at few distinct processing positions for a profile
  // with its extremum at the pencil's centre and zero ghost cells at both
  // ends: segment 2 (starting at the centre) fails at its first two faces,
  // segment 0 (inflow) at its first, segment 1 (ending at the centre) at its
  // last, segment 3 (outflow) rarely.  Which lane computes which
  // (segment, pencil) does not change any result.
  const int sl = tid / PN;
  const int s = S == 4 ? (0x1302 >> (4 * sl)) & 15 : sl;
  const int u = tid - sl * PN;
  const int cq = u / N;
  const int cj = u - cq * N;
  const int m0 = s * R;
  const T* colA = lds + cq * PS + G * P + G + cj;    // along v_{D-1}: stride P
  const T* colB = lds + cq * PS + (G + cj) * P + G;  // along v_D: stride 1

  V pf[NV];
  // several runs of one geometry (batched ensembles): tile tt belongs to
  // run tt / tpr with f fmulti[r] and tables tmulti[r] (v_{D-1}) and
  // tmulti[nrun + r] (v_D); pl.planes counts the planes of one run
  const int64_t nrun = a.fmulti ? pl.tiles / a.tpr : 1;
  int np_next = 0;
  int64_t p0_next = 0;
  T* f_next = f;
  const PencilEntry<T>* ta_next = tabA;
  const PencilEntry<T>* tb_next = tabB;
  auto issue = [&](int64_t tt) __attribute__((always_inline)) {
    int64_t lt = tt;
    ta_next = tabA;
    tb_next = tabB;
    if (a.fmulti) {
      const int64_t r = tt / a.tpr;
      lt = tt - r * a.tpr;
      f_next = reinterpret_cast<T*>(load_ptr_uniform(a.fmulti + r));
      ta_next = reinterpret_cast<const PencilEntry<T>*>(load_ptr_uniform(a.tmulti + r));
      tb_next = reinterpret_cast<const PencilEntry<T>*>(load_ptr_uniform(a.tmulti + nrun + r));
    }
    p0_next = lt * PB;
    np_next = (int)min<int64_t>(PB, pl.planes - p0_next);
    const V* src = reinterpret_cast<const V*>(f_next + p0_next * NN);
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (vq[k] < np_next) pf[k] = __builtin_nontemporal_load(src + tid + NT * k);
  };
  int64_t t = blockIdx.x;
  if (t < pl.tiles) issue(t);
  for (; t < pl.tiles; t += gridDim.x) {
    const int np = np_next;
    const int64_t p0 = p0_next;
    T* const fc = f_next;
    const bool act = cq < np;
    // the two pencil entries of this thread's plane (with UNI: of every
    // plane of the tile, read with scalar loads), requested before the
    // tile's data go to LDS
    PencilEntry<T> eA{}, eB{};
    if (UNI || act) {
      const int64_t pp = UNI ? p0 : p0 + cq;
      const int64_t ix = pl.vdiv.m ? (int64_t)pl.vdiv.div((uint32_t)pp) : udiv(pp, pl.vouter);
      eA = load_entry_uniform(ta_next + ix);
      eB = load_entry_uniform(tb_next + ix);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (vq[k] < np) put(lds + loff[k], pf[k]);
    __syncthreads();
    if (t + gridDim.x < pl.tiles) issue(t + gridDim.x);
    T out[R];
    // v_{D-1}
    if (act) {
      if (eA.absN <= kPlaneFast) {
        if (eA.dir > 0)
          advance_ct<T, ORDER, R, P, 1>(colA, eA, m0, alpha, out);
        else
          advance_ct<T, ORDER, R, P, -1>(colA, eA, m0, alpha, out);
      } else {
        advance<T, ORDER, SLMPP_LIM_MPP, READ_SAFE, R>(colA, P, N, G, 0, eA, m0, R, alpha, out,
                                                        nullptr);
      }
    }
    __syncthreads();
    if (act) {
      if (eA.dir > 0)
        store_ct<T, R, P, 1>(const_cast<T*>(colA), N, m0, out);
      else
        store_ct<T, R, P, -1>(const_cast<T*>(colA), N, m0, out);
    }
    __syncthreads();
    // v_D on the updated plane
    if (act) {
      if (eB.absN <= kPlaneFast) {
        if (eB.dir > 0)
          advance_ct<T, ORDER, R, 1, 1>(colB, eB, m0, alpha, out);
        else
          advance_ct<T, ORDER, R, 1, -1>(colB, eB, m0, alpha, out);
      } else {
        advance<T, ORDER, SLMPP_LIM_MPP, READ_SAFE, R>(colB, 1, N, G, 0, eB, m0, R, alpha, out,
                                                        nullptr);
      }
    }
    __syncthreads();
    if (act) {
      if (eB.dir > 0)
        store_ct<T, R, 1, 1>(const_cast<T*>(colB), N, m0, out);
      else
        store_ct<T, R, 1, -1>(const_cast<T*>(colB), N, m0, out);
    }
    __syncthreads();
    V* dst = reinterpret_cast<V*>(fc + p0 * NN);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if (vq[k] < np) {
        V v;
        get(lds + loff[k], v);
        __builtin_nontemporal_store(v, dst + tid + NT * k);
      }
    }
    // no barrier before the next tile: its first LDS writes are this
    // thread's own data-movement vectors, at the offsets it has just read
  }
}

// Pencil-table entry for speed index idx (see PencilEntry).
template <typename T, int ORDER>
__device__ __forceinline__ PencilEntry<T> pencil_entry(const SweepArgs& a, int idx) {
  const double c = a.cmode == SPEED_FROM_VELOCITY ? cell_center(a.vlo, a.dv, idx) : a.accel[idx];
  const double xi = departure(c, a.dt, a.h);
  const int n = a.n;
  double zeta;
  int64_t N;
  if (a.rk) {
    // TVD-RK stage (Sec. 2.1.1): no shift, the CFL number itself as zeta;
    // |nu| > 1 poisons the pencil
    N = 0;
    zeta = fabs(xi) <= 1.0 ? xi : __builtin_nan("");
  } else if (!(fabs(xi) < 4.0e18)) {  // non-finite or absurd offset: poison the pencil
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
  PencilEntry<T> e{};
  e.dir = mirror ? -1 : 1;
  e.base = (int32_t)((mirror ? (int64_t)(n - 1) : 0) - N);
  e.absN = (int16_t)(N < 0 ? -N : N);
  e.z = (T)az;
  e.tz = (T)(az + az);
  // an RK stage takes the interface interpolation itself: the flux
  // polynomial at zero Courant number
  const double zw = a.rk ? 0.0 : az;
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
      acc = acc * zw + fr.num / fr.den;
    }
    e.w[k] = (T)acc;
  }
  return e;
}

template <typename T, int ORDER>
__global__ void pencil_table_kernel(SweepArgs a, PencilEntry<T>* __restrict__ tab, int count) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) tab[idx] = pencil_entry<T, ORDER>(a, idx);
}

size_t entry_bytes(int dtype) {
  return dtype == SLMPP_F64 ? sizeof(PencilEntry<double>) : sizeof(PencilEntry<float>);
}

template <typename T, int ORDER, int LIM, int RC, int WT>
hipError_t launch_k(const SweepArgs& a, const SweepPlan& p, const void* table, hipStream_t s) {
  auto kern = sweep_kernel<T, ORDER, LIM, RC, WT>;
  if (p.lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)p.tiles), dim3(p.threads), p.lds_bytes, s, a, p,
                     reinterpret_cast<const PencilEntry<T>*>(table));
  return hipGetLastError();
}

template <typename T, int ORDER, int RC, int WT, bool CONTIG, bool MOM = false>
hipError_t launch_fast(const SweepArgs& a, const SweepPlan& p, const void* table, hipStream_t s) {
  auto kern = sweep_fast_kernel<T, ORDER, RC, WT, CONTIG, MOM>;
  if (p.lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(kern), p.threads, p.lds_bytes);
  if (e != hipSuccess) return e;
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  const int64_t slots = (int64_t)std::max(per_cu, 1) * std::max(n_cu, 1);
  const int64_t grid = std::min<int64_t>(p.tiles, slots);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(p.threads), p.lds_bytes, s, a, p,
                     reinterpret_cast<const PencilEntry<T>*>(table));
  return hipGetLastError();
}

template <typename T, int ORDER, int RC>
hipError_t launch_w(const SweepArgs& a, const SweepPlan& p, const void* table, hipStream_t s) {
  if constexpr (RC == 32) {  // strided 128-pencil tiles of 64-cell pencils only
    if (!p.fast || a.inner == 1 || p.W != 128) return hipErrorInvalidValue;
    if (a.mom) return launch_fast<T, ORDER, RC, 128, false, true>(a, p, table, s);
    return launch_fast<T, ORDER, RC, 128, false>(a, p, table, s);
  } else {
    if (p.fast) {
      if (a.inner == 1) return launch_fast<T, ORDER, RC, 64, true>(a, p, table, s);
      switch (p.W) {
        case 256:
          if constexpr (RC == 24 && ORDER == 7 && sizeof(T) == 4) {
            if (a.mom) return launch_fast<T, ORDER, RC, 256, false, true>(a, p, table, s);
            return launch_fast<T, ORDER, RC, 256, false>(a, p, table, s);
          }
          break;
        case 128:
          if (a.mom) return launch_fast<T, ORDER, RC, 128, false, true>(a, p, table, s);
          return launch_fast<T, ORDER, RC, 128, false>(a, p, table, s);
        case 64:
          if (a.mom) return launch_fast<T, ORDER, RC, 64, false, true>(a, p, table, s);
          return launch_fast<T, ORDER, RC, 64, false>(a, p, table, s);
        case 48: return launch_fast<T, ORDER, RC, 48, false>(a, p, table, s);
        case 32: return launch_fast<T, ORDER, RC, 32, false>(a, p, table, s);
        default: break;
      }
    }
    return launch_k<T, ORDER, SLMPP_LIM_MPP, RC, 0>(a, p, table, s);
  }
}

template <typename T, int ORDER, int LIM>
hipError_t launch_r(const SweepArgs& a, const SweepPlan& p, const void* table, hipStream_t s) {
  if constexpr (LIM == SLMPP_LIM_MPP) {
    switch (p.R) {
      case 12: return launch_w<T, ORDER, 12>(a, p, table, s);
      case 16: return launch_w<T, ORDER, 16>(a, p, table, s);
      case 24: return launch_w<T, ORDER, 24>(a, p, table, s);
      case 32:  // planned for FP32 only
        if constexpr (sizeof(T) == 4) return launch_w<T, ORDER, 32>(a, p, table, s);
        return hipErrorInvalidValue;
      default: break;
    }
  }
  SweepPlan g = p;
  g.R = 0;
  return launch_k<T, ORDER, LIM, 0, 0>(a, g, table, s);
}

template <typename T, int ORDER>
hipError_t launch_o(int limiter, const SweepArgs& a, const SweepPlan& p, const void* table,
                    hipStream_t s) {
  if (p.tiles <= 0) return hipSuccess;
  switch (limiter) {
    case SLMPP_LIM_NONE: return launch_r<T, ORDER, SLMPP_LIM_NONE>(a, p, table, s);
    case SLMPP_LIM_MP: return launch_r<T, ORDER, SLMPP_LIM_MP>(a, p, table, s);
    default: return launch_r<T, ORDER, SLMPP_LIM_MPP>(a, p, table, s);
  }
}

template <typename T, int ORDER>
hipError_t launch_table_t(const SweepArgs& a, void* table, int count, hipStream_t s) {
  hipLaunchKernelGGL((pencil_table_kernel<T, ORDER>), dim3((count + 127) / 128), dim3(128), 0, s,
                     a, reinterpret_cast<PencilEntry<T>*>(table), count);
  return hipGetLastError();
}

// ---- grouped launches over many independent runs ----------------------
template <typename T>
__global__ void batch_table_kernel(const BatchSweep* __restrict__ sweeps) {
  const BatchSweep& b = sweeps[blockIdx.y];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= b.count) return;
  PencilEntry<T>* tab = reinterpret_cast<PencilEntry<T>*>(b.table);
  tab[idx] = b.order == 7 ? pencil_entry<T, 7>(b.a, idx) : pencil_entry<T, 5>(b.a, idx);
}

// Persistent over work items; every item is one tile of one run's sweep,
// with its own shape, plan (256 threads) and order.  Segments of 8, 12 or
// 16 cells per thread (pl.R) take the compile-time variants, which keep a
// segment's outputs in registers; other lengths take the runtime one.
template <typename T>
__global__ void __launch_bounds__(256) batch_sweep_kernel(const BatchSweep* __restrict__ sweeps,
                                                          const BatchItem* __restrict__ items,
                                                          int nitems) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchItem item = items[it];
    const BatchSweep& b = sweeps[item.sweep];
    const SweepArgs a = b.a;
    const SweepPlan pl = b.p;
    const PencilEntry<T>* tab = reinterpret_cast<const PencilEntry<T>*>(b.table);
    const int64_t t = item.tile;
    switch (b.order * 100 + pl.R) {
      case 508: sweep_tile<T, 5, SLMPP_LIM_MPP, 8, 0, false>(a, pl, tab, t, smem); break;
      case 512: sweep_tile<T, 5, SLMPP_LIM_MPP, 12, 0, false>(a, pl, tab, t, smem); break;
      case 516: sweep_tile<T, 5, SLMPP_LIM_MPP, 16, 0, false>(a, pl, tab, t, smem); break;
      case 708: sweep_tile<T, 7, SLMPP_LIM_MPP, 8, 0, false>(a, pl, tab, t, smem); break;
      case 712: sweep_tile<T, 7, SLMPP_LIM_MPP, 12, 0, false>(a, pl, tab, t, smem); break;
      case 716: sweep_tile<T, 7, SLMPP_LIM_MPP, 16, 0, false>(a, pl, tab, t, smem); break;
      case 700: sweep_tile<T, 7, SLMPP_LIM_MPP, 0, 0, false>(a, pl, tab, t, smem); break;
      default: sweep_tile<T, 5, SLMPP_LIM_MPP, 0, 0, false>(a, pl, tab, t, smem); break;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_batch_tables(int dtype, const BatchSweep* sweeps, int nsweeps, int max_count,
                               hipStream_t s) {
  if (nsweeps <= 0 || max_count <= 0) return hipSuccess;
  const dim3 grid((max_count + 127) / 128, nsweeps);
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(batch_table_kernel<double>, grid, dim3(128), 0, s, sweeps);
  else
    hipLaunchKernelGGL(batch_table_kernel<float>, grid, dim3(128), 0, s, sweeps);
  return hipGetLastError();
}

hipError_t prepare_batch_sweep(int dtype, size_t lds_bytes) {
  const void* k = dtype == SLMPP_F64 ? reinterpret_cast<const void*>(batch_sweep_kernel<double>)
                                     : reinterpret_cast<const void*>(batch_sweep_kernel<float>);
  if (lds_bytes > 64 * 1024)
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  return hipSuccess;
}

int batch_sweep_blocks_per_cu(int dtype, size_t lds_bytes) {
  int per_cu = 0;
  const void* k = dtype == SLMPP_F64 ? reinterpret_cast<const void*>(batch_sweep_kernel<double>)
                                     : reinterpret_cast<const void*>(batch_sweep_kernel<float>);
  if (lds_bytes > 64 * 1024)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds_bytes) != hipSuccess)
    return 1;
  return per_cu > 0 ? per_cu : 1;
}

hipError_t launch_batch_sweeps(int dtype, const BatchSweep* sweeps, const BatchItem* items,
                               int nitems, size_t lds_bytes, int grid, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(batch_sweep_kernel<double>, dim3(grid), dim3(256), lds_bytes, s, sweeps,
                       items, nitems);
  else
    hipLaunchKernelGGL(batch_sweep_kernel<float>, dim3(grid), dim3(256), lds_bytes, s, sweeps,
                       items, nitems);
  return hipGetLastError();
}

hipError_t launch_generic_sweep(int dtype, int order, const SweepArgs& a, const SweepPlan& p,
                                const void* table, hipStream_t s) {
  SweepPlan g = p;
  g.R = 0;
  g.fast = 0;
  if (dtype == SLMPP_F64)
    return order == 7 ? launch_k<double, 7, SLMPP_LIM_MPP, 0, 0>(a, g, table, s)
                      : launch_k<double, 5, SLMPP_LIM_MPP, 0, 0>(a, g, table, s);
  return order == 7 ? launch_k<float, 7, SLMPP_LIM_MPP, 0, 0>(a, g, table, s)
                    : launch_k<float, 5, SLMPP_LIM_MPP, 0, 0>(a, g, table, s);
}

namespace {
size_t entry_bytes_any(int dtype) { return entry_bytes(dtype); }
}  // namespace

// Plan of a batch sweep: 256 threads, W pencils per tile (W * S = 256).
// A pencil length n = S * R with R in {8, 12, 16} takes the register
// variant (R); others the runtime segment length (R = 0), which also keeps
// its outputs in a second LDS tile.  lds_bytes == 0: the tile does not fit
// kBatchTileLdsMax.
SweepPlan plan_batch_sweep(int dtype, int order, int32_t n, int64_t npen, int64_t inner,
                           int32_t nfast, int W) {
  SweepPlan p{};
  const size_t es = dtype == SLMPP_F64 ? 8 : 4;
  const int gh = order == 7 ? 4 : 3;
  p.G = gh + nfast;
  const bool contiguous = inner == 1;
  int P = n + 2 * p.G;
  if ((P & 1) == 0) ++P;
  p.pitch = contiguous ? P : W;
  p.W = W;
  p.S = 256 / W;
  p.threads = 256;
  const int R = n % p.S == 0 ? n / p.S : 0;
  p.R = (R == 8 || R == 12 || R == 16) ? R : 0;
  const size_t elems = contiguous ? (size_t)W * P : (size_t)(n + 2 * p.G) * W;
  size_t b = (elems * es + 15) & ~(size_t)15;
  b += (size_t)W * entry_bytes_any(dtype);
  if (p.R == 0) b += elems * es;
  p.lds_bytes = b <= kBatchTileLdsMax ? b : 0;
  p.tiles = (npen + W - 1) / W;
  p.fast = 0;
  return p;
}


size_t pencil_table_bytes(int dtype, int64_t count) { return entry_bytes(dtype) * (size_t)count; }

SweepPlan plan_sweep(int dtype, int order, int limiter, int32_t n, int64_t npen, int64_t inner,
                     int32_t nfast, int W_override, int S_override, bool moment) {
  SweepPlan p{};
  const size_t es = dtype == SLMPP_F64 ? 8 : 4;
  const int gh = order == 7 ? 4 : 3;
  p.G = gh + nfast;
  const bool contiguous = inner == 1;
  auto pitch_of = [&](int W) {
    (void)W;
    int P = n + 2 * p.G;  // contiguous: pencil-major rows, odd pitch
    if ((P & 1) == 0) ++P;
    return contiguous ? P : W;
  };
  auto lds = [&](int W, bool regs) {
    const size_t elems = contiguous ? (size_t)W * pitch_of(W) : (size_t)(n + 2 * p.G) * W;
    size_t b = (elems * es + 15) & ~(size_t)15;
    b += (size_t)W * entry_bytes(dtype);
    if (!regs) b += elems * es;
    return b;
  };
  // W: pencils per tile.  Strided tiles should not straddle a block of
  // `inner` pencils, so W divides inner when a divisor in the list exists.
  // Wider tiles read longer contiguous runs of each row (128 pencils: 512 B
  // in FP32), which the strided x sweeps need; a width is taken only when
  // some compile-time segment length fits it.  Segments of 32 cells exist
  // only for strided 128-pencil tiles of 64-cell FP32 pencils, and not with
  // the row sums of the moment: with those, or in FP64, their registers
  // would halve the occupancy, and 64-pencil tiles of 16-cell segments are
  // faster.
  auto seg_ok = [&](int c, int Wc) {
    return n % c == 0 && Wc * (n / c) <= 256 &&
           (c != 32 || (Wc == 128 && n == 64 && !contiguous && !moment && es == 4));
  };
  auto has_r = [&](int Wc) {
    for (int c : {12, 16, 24, 32})
      if (seg_ok(c, Wc)) return true;
    return false;
  };
  int W = 0;
  if (W_override > 0) {
    W = W_override;
  } else if (contiguous) {
    W = 64;
  } else {
    for (int c : {128, 64, 48, 32, 16}) {
      if (inner % c == 0 && has_r(c)) {
        W = c;
        break;
      }
    }
    if (W == 0) {
      for (int c : {64, 48, 32, 16}) {
        if (inner % c == 0) {
          W = c;
          break;
        }
      }
    }
    if (W == 0) W = 64;
  }
  while (W > 1 && lds(W, false) > 96 * 1024) W /= 2;
  // 48-cell strided SL-MPP7 pencils take tiles of two 24-cell segments,
  // 256 pencils wide in FP32 (see sweep_fast_kernel) and 128 in FP64 (two
  // such workgroups fit a CU in registers and LDS, with 1 KiB per row)
  const bool wide = !contiguous && n == 48 && order == 7 && inner % (es == 4 ? 256 : 128) == 0 &&
                    W_override == 0 && S_override <= 0 && limiter == SLMPP_LIM_MPP;
  if (wide) W = es == 4 ? 256 : 128;
  // R: cells per thread; a compile-time length when it divides n
  int R = 0;
  if (S_override > 0) {
    const int S = S_override;
    R = (n % S == 0 && (n / S == 12 || n / S == 16 || n / S == 24)) ? n / S : 0;
    p.S = S;
  } else {
    for (int c : {12, 16, 24, 32}) {
      if (seg_ok(c, W)) {
        R = c;
        break;
      }
    }
    p.S = R ? n / R : std::max(1, std::min(256 / std::max(1, W), std::max(1, n / 8)));
  }
  p.S = std::max(1, std::min(p.S, 256 / std::max(1, W)));
  if (wide) {
    R = 24;
    p.S = 2;
  }
  if (R && p.S * R != n) R = 0;
  if (limiter != SLMPP_LIM_MPP) R = 0;  // compile-time segments exist for SL-MPP only
  p.R = R;
  p.W = W;
  p.threads = W * p.S;
  p.pitch = pitch_of(W);
  p.lds_bytes = lds(W, R > 0);
  p.tiles = (npen + W - 1) / W;
  // the persistent prefetching kernel (see sweep_fast_kernel)
  const int vn = dtype == SLMPP_F64 ? 2 : 4;
  const bool fits32 = npen < ((int64_t)1 << 31) && inner < ((int64_t)1 << 31) &&
                      (int64_t)n * W < ((int64_t)1 << 24);
  p.fast = R > 0 && R % vn == 0 && fits32 && W_override == 0 &&
           (contiguous ? (W == 64 && n % vn == 0) : (inner % W == 0 && inner % vn == 0 &&
                                                     (W == 256 || W == 128 || W == 64 || W == 48 || W == 32)));
  if (R == 32 && !p.fast) {  // 32-cell segments exist in the fast kernel only
    R = 0;
    p.R = 0;
    p.lds_bytes = lds(W, false);
  }
  if (p.fast) p.lds_bytes = lds(W, true);
  return p;
}

hipError_t launch_pencil_table(int dtype, int order, const SweepArgs& a, void* table,
                               int64_t table_count, hipStream_t s) {
  const int count = (int)table_count;
  if (dtype == SLMPP_F64)
    return order == 7 ? launch_table_t<double, 7>(a, table, count, s)
                      : launch_table_t<double, 5>(a, table, count, s);
  return order == 7 ? launch_table_t<float, 7>(a, table, count, s)
                    : launch_table_t<float, 5>(a, table, count, s);
}

hipError_t launch_sweep(int dtype, int order, int limiter, const SweepArgs& a, const SweepPlan& p,
                        const void* table, hipStream_t s) {
  if (dtype == SLMPP_F64)
    return order == 7 ? launch_o<double, 7>(limiter, a, p, table, s)
                      : launch_o<double, 5>(limiter, a, p, table, s);
  return order == 7 ? launch_o<float, 7>(limiter, a, p, table, s)
                    : launch_o<float, 5>(limiter, a, p, table, s);
}

namespace {
template <typename T, int ORDER, int N, bool UNI>
hipError_t launch_plane_u(const SweepArgs& a, const PlanePlan& p, const void* tabA,
                          const void* tabB, hipStream_t s) {
  auto kern = kick_plane_kernel<T, ORDER, N, UNI>;
  if (p.lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)p.lds_bytes);
    if (e != hipSuccess) return e;
  }
  constexpr int NT = PlaneShape<T, ORDER, N>::threads;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(kern), NT, p.lds_bytes);
  if (e != hipSuccess) return e;
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  const int64_t grid = std::min<int64_t>(p.tiles, (int64_t)std::max(per_cu, 1) * std::max(n_cu, 1));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), p.lds_bytes, s, a, p,
                     reinterpret_cast<const PencilEntry<T>*>(tabA),
                     reinterpret_cast<const PencilEntry<T>*>(tabB));
  return hipGetLastError();
}

template <typename T, int ORDER, int N>
hipError_t launch_plane_t(const SweepArgs& a, const PlanePlan& p, const void* tabA,
                          const void* tabB, hipStream_t s) {
  return p.uni ? launch_plane_u<T, ORDER, N, true>(a, p, tabA, tabB, s)
               : launch_plane_u<T, ORDER, N, false>(a, p, tabA, tabB, s);
}

template <typename T, int ORDER>
hipError_t launch_plane_o(const SweepArgs& a, const PlanePlan& p, const void* tabA,
                          const void* tabB, hipStream_t s) {
  switch (p.N) {
    case 24: return launch_plane_t<T, ORDER, 24>(a, p, tabA, tabB, s);
    case 32: return launch_plane_t<T, ORDER, 32>(a, p, tabA, tabB, s);
    case 48: return launch_plane_t<T, ORDER, 48>(a, p, tabA, tabB, s);
    case 64: return launch_plane_t<T, ORDER, 64>(a, p, tabA, tabB, s);
    default: return hipErrorInvalidValue;
  }
}

// the host's copy of PlaneShape
template <typename T, int ORDER, int N>
void plane_shape(PlanePlan& p) {
  using Sh = PlaneShape<T, ORDER, N>;
  p.N = N;
  p.PB = Sh::PB;
  p.G = Sh::G;
  p.pitch = Sh::P;
  p.plane_lds = Sh::PS;
}
template <typename T, int ORDER>
bool plane_shape_n(int N, PlanePlan& p) {
  switch (N) {
    case 24: plane_shape<T, ORDER, 24>(p); return true;
    case 32: plane_shape<T, ORDER, 32>(p); return true;
    case 48: plane_shape<T, ORDER, 48>(p); return true;
    case 64: plane_shape<T, ORDER, 64>(p); return true;
    default: return false;
  }
}
}  // namespace

PlanePlan plan_kick_plane(int dtype, int order, int32_t na, int32_t nb, int64_t planes,
                          int64_t vouter) {
  PlanePlan p{};
  if (na != nb || !(na == 24 || na == 32 || na == 48 || na == 64) || planes < 1 || vouter < 1)
    return p;
  const bool ok = dtype == SLMPP_F64
                      ? (order == 7 ? plane_shape_n<double, 7>(na, p) : plane_shape_n<double, 5>(na, p))
                      : (order == 7 ? plane_shape_n<float, 7>(na, p) : plane_shape_n<float, 5>(na, p));
  if (!ok) return PlanePlan{};
  p.planes = planes;
  p.vouter = vouter;
  p.tiles = (planes + p.PB - 1) / p.PB;
  // every tile's planes belong to one spatial cell: one pair of entries
  p.uni = vouter % p.PB == 0 ? 1 : 0;
  if (planes < ((int64_t)1 << 32) && vouter < ((int64_t)1 << 31)) p.vdiv = FastDiv32::of((uint32_t)vouter);
  const size_t es = dtype == SLMPP_F64 ? 8 : 4;
  const size_t lds = ((size_t)p.PB * p.plane_lds * es + 15) & ~(size_t)15;  // entries: registers
  p.lds_bytes = lds <= 80 * 1024 ? lds : 0;
  return p;
}

hipError_t launch_kick_plane(int dtype, int order, const SweepArgs& a, const PlanePlan& p,
                             const void* tabA, const void* tabB, hipStream_t s) {
  if (p.lds_bytes == 0) return hipErrorInvalidValue;
  if (dtype == SLMPP_F64)
    return order == 7 ? launch_plane_o<double, 7>(a, p, tabA, tabB, s)
                      : launch_plane_o<double, 5>(a, p, tabA, tabB, s);
  return order == 7 ? launch_plane_o<float, 7>(a, p, tabA, tabB, s)
                    : launch_plane_o<float, 5>(a, p, tabA, tabB, s);
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
