// Field kernels: velocity moment, periodic Poisson solve with high-order
// Green functions and forces (Sec. 2.2, App. C), initialisation, and
// reductions for diagnostics.  All field arithmetic is double precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "slmpp_internal.hpp"

namespace slmpp {
namespace {

// ---- compensated (Neumaier) accumulation ------------------------------
struct KSum {
  double s, c;
};
__device__ __forceinline__ void kadd(KSum& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ void kmerge(KSum& a, const KSum& b) {
  kadd(a, b.s);
  a.c += b.c;
}

template <int NT>
__device__ KSum block_ksum(KSum v) {
  __shared__ double ss[NT], sc[NT];
  ss[threadIdx.x] = v.s;
  sc[threadIdx.x] = v.c;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      KSum a{ss[threadIdx.x], sc[threadIdx.x]};
      KSum b{ss[threadIdx.x + off], sc[threadIdx.x + off]};
      kmerge(a, b);
      ss[threadIdx.x] = a.s;
      sc[threadIdx.x] = a.c;
    }
    __syncthreads();
  }
  KSum r{ss[0], sc[0]};
  __syncthreads();
  return r;
}

// rho[ix] = dvol * sum over the contiguous velocity block of cell ix.
// One workgroup per spatial cell; fixed reduction order (deterministic).
// When the block is a whole number of 16-byte vectors, each thread reads
// vectors (four loads in flight), adds a vector's components in double and
// feeds the sum to one of two compensated accumulators.
template <typename T>
struct MomVec;
template <>
struct MomVec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
  __device__ static double sum(type v) {
    return ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
  }
};
template <>
struct MomVec<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
  __device__ static double sum(type v) { return v.x + v.y; }
};

template <typename T, int NT>
__global__ void __launch_bounds__(NT) moment_kernel(const T* __restrict__ f, int64_t nvs,
                                                    double dvol, double* __restrict__ rho) {
  using MV = MomVec<T>;
  using V = typename MV::type;
  const T* b = f + (int64_t)blockIdx.x * nvs;
  KSum acc0{0.0, 0.0}, acc1{0.0, 0.0};
  if (nvs % MV::N == 0) {
    const V* bv = reinterpret_cast<const V*>(b);
    const int64_t nv = nvs / MV::N;
    constexpr int U = 4;
    int64_t k = threadIdx.x;
    for (; k + (U - 1) * NT < nv; k += U * NT) {
      V x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = bv[k + u * NT];
#pragma unroll
      for (int u = 0; u < U; u += 2) {
        kadd(acc0, MV::sum(x[u]));
        kadd(acc1, MV::sum(x[u + 1]));
      }
    }
    for (; k < nv; k += NT) kadd(acc0, MV::sum(bv[k]));
  } else {
    for (int64_t k = threadIdx.x; k < nvs; k += NT) kadd(acc0, (double)b[k]);
  }
  kmerge(acc0, acc1);
  KSum tot = block_ksum<NT>(acc0);
  if (threadIdx.x == 0) rho[blockIdx.x] = dvol * (tot.s + tot.c);
}

// Velocity moments of one spatial cell per workgroup (Sec. 2.3): density,
// mean velocity and dispersion per velocity axis, two passes over the
// cell's contiguous velocity block (the second re-reads it from cache);
// compensated double sums of plain sums over groups of eight elements.
template <typename T, int NT, int D>  // D: velocity axes (a constant: the loops over
                                      // axes unroll and every accumulator stays in registers)
__global__ void __launch_bounds__(NT) velocity_moments_kernel(const T* __restrict__ f, int,
                                                              int64_t nvs, int3 nv, double3 vlo,
                                                              double3 dv, double dvol, int64_t nxs,
                                                              double* __restrict__ rho,
                                                              double* __restrict__ mean,
                                                              double* __restrict__ disp) {
  const T* b = f + (int64_t)blockIdx.x * nvs;
  const int n[3] = {nv.x, nv.y, nv.z};
  const double lo[3] = {vlo.x, vlo.y, vlo.z}, h[3] = {dv.x, dv.y, dv.z};
  // velocity index of element k as digits (last axis fastest): the digits
  // of this thread's first element and of the stride NT, then a digit-wise
  // add with carries per step instead of a division per element
  int j0[3] = {0, 0, 0}, st[3] = {0, 0, 0};
  {
    int64_t rem = threadIdx.x, str = NT;
    for (int l = D - 1; l >= 0; --l) {
      j0[l] = (int)(rem % n[l]);
      rem /= n[l];
      st[l] = (int)(str % n[l]);
      str /= n[l];
    }
  }
  int j[3];
  auto restart = [&]() {
    for (int l = 0; l < 3; ++l) j[l] = j0[l];
  };
  auto centres = [&](double* v) {
    for (int l = 0; l < D; ++l) v[l] = lo[l] + ((double)j[l] + 0.5) * h[l];
  };
  auto next = [&]() {  // j += st; past the last element the digits are unused
    int carry = 0;
    for (int l = D - 1; l >= 0; --l) {
      j[l] += st[l] + carry;
      carry = j[l] >= n[l];
      if (carry) j[l] -= n[l];
    }
  };
  // each thread adds groups of up to kGroup of its elements plainly and
  // feeds the group sums to the compensated accumulators
  constexpr int kGroup = 8;
  KSum s0{0.0, 0.0}, s1[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  double p0 = 0.0, p1[3] = {0.0, 0.0, 0.0};
  int cnt = 0;
  restart();
  for (int64_t k = threadIdx.x; k < nvs; k += NT, next()) {
    double v[3];
    centres(v);
    const double x = (double)b[k];
    p0 += x;
    for (int l = 0; l < D; ++l) p1[l] += x * v[l];
    if (++cnt == kGroup) {
      kadd(s0, p0);
      for (int l = 0; l < D; ++l) kadd(s1[l], p1[l]);
      p0 = 0.0;
      for (int l = 0; l < D; ++l) p1[l] = 0.0;
      cnt = 0;
    }
  }
  kadd(s0, p0);
  for (int l = 0; l < D; ++l) kadd(s1[l], p1[l]);
  const KSum t0 = block_ksum<NT>(s0);
  const double m0 = t0.s + t0.c;
  double u[3] = {0.0, 0.0, 0.0};
  for (int l = 0; l < D; ++l) {
    const KSum t1 = block_ksum<NT>(s1[l]);
    u[l] = m0 != 0.0 ? (t1.s + t1.c) / m0 : 0.0;
  }
  KSum s2[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  double p2[3] = {0.0, 0.0, 0.0};
  cnt = 0;
  restart();
  for (int64_t k = threadIdx.x; k < nvs; k += NT, next()) {
    double v[3];
    centres(v);
    const double x = (double)b[k];
    for (int l = 0; l < D; ++l) {
      const double d = v[l] - u[l];
      p2[l] += x * d * d;
    }
    if (++cnt == kGroup) {
      for (int l = 0; l < D; ++l) {
        kadd(s2[l], p2[l]);
        p2[l] = 0.0;
      }
      cnt = 0;
    }
  }
  for (int l = 0; l < D; ++l) kadd(s2[l], p2[l]);
  for (int l = 0; l < D; ++l) {
    const KSum t2 = block_ksum<NT>(s2[l]);
    if (threadIdx.x == 0) {
      mean[(int64_t)l * nxs + blockIdx.x] = u[l];
      disp[(int64_t)l * nxs + blockIdx.x] = m0 != 0.0 ? (t2.s + t2.c) / m0 : 0.0;
    }
  }
  if (threadIdx.x == 0) rho[blockIdx.x] = dvol * m0;
}

// F[k] = xvol * sum_x f[x][k]: one thread per velocity cell.  Few threads
// walk long columns here (one per velocity cell), so each keeps 16 loads in
// flight: rows x = 16 m + r go to accumulator r % 4, merged in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) velocity_distribution_kernel(const T* __restrict__ f,
                                                                    int64_t nxs, int64_t nvs,
                                                                    double xvol,
                                                                    double* __restrict__ F) {
  constexpr int U = 16;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvs;
       k += (int64_t)gridDim.x * blockDim.x) {
    KSum a[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    const T* col = f + k;
    int64_t ix = 0;
    for (; ix + U <= nxs; ix += U) {
      T x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = col[(ix + u) * nvs];
#pragma unroll
      for (int u = 0; u < U; ++u) kadd(a[u % 4], (double)x[u]);
    }
    for (; ix < nxs; ++ix) kadd(a[0], (double)col[ix * nvs]);
    kmerge(a[0], a[1]);
    kmerge(a[2], a[3]);
    kmerge(a[0], a[2]);
    F[k] = xvol * (a[0].s + a[0].c);
  }
}

// rho[i * ncol + c] = dvol * sum_q part[(c * nsub + q) * n + i]; thread
// (c, i) adds the nsub tile-row sums of its cell in tile order (compensated).
__global__ void __launch_bounds__(256) moment_reduce_kernel(const double* __restrict__ part, int n,
                                                            int64_t ncol, int64_t nsub, double dvol,
                                                            double* __restrict__ rho) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncol * n) return;
  const int64_t c = g / n;
  const int i = (int)(g - c * n);
  const double* p = part + c * nsub * n + i;
  KSum acc0{0.0, 0.0}, acc1{0.0, 0.0};
  int64_t q = 0;
  for (; q + 1 < nsub; q += 2) {
    const double x0 = p[q * n], x1 = p[(q + 1) * n];
    kadd(acc0, x0);
    kadd(acc1, x1);
  }
  if (q < nsub) kadd(acc0, p[q * n]);
  kmerge(acc0, acc1);
  rho[(int64_t)i * ncol + c] = dvol * (acc0.s + acc0.c);
}

// ---- discrete Fourier transform along one axis ------------------------
// out[o, k, j] = sum_m in[o, m, j] * tw[(m k) mod n]^sign, tw[q] = exp(-2 pi i q / n)
__global__ void dft_axis_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                int64_t total, int64_t n, int64_t inner,
                                const double2* __restrict__ tw, int conj) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t j = t % inner;
  const int64_t k = (t / inner) % n;
  const int64_t o = t / (inner * n);
  const double2* src = in + o * n * inner + j;
  double sr = 0.0, si = 0.0;
  int64_t q = 0;
  for (int64_t m = 0; m < n; ++m) {
    const double2 x = src[m * inner];
    const double2 w = tw[q];
    const double wi = conj ? -w.y : w.y;
    sr += x.x * w.x - x.y * wi;
    si += x.x * wi + x.y * w.x;
    q += k;
    if (q >= n) q -= n;
  }
  out[t] = make_double2(sr, si);
}

__global__ void real_to_complex_kernel(const double* __restrict__ r, double2* __restrict__ c,
                                       int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) c[t] = make_double2(r[t], 0.0);
}

__global__ void green_kernel(double2* __restrict__ c, const double* __restrict__ g, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    const double2 v = c[t];
    c[t] = make_double2(v.x * g[t], v.y * g[t]);
  }
}

__global__ void complex_to_real_kernel(const double2* __restrict__ c, double* __restrict__ r,
                                       int64_t n, double scale) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) r[t] = c[t].x * scale;
}

// accel_l = -dphi/dx_l by the periodic 2-, 4- or 6-point FDA (App. C)
__global__ void fda_kernel(const double* __restrict__ phi, double* __restrict__ accel,
                           int64_t total, int64_t n, int64_t inner, double h, int order) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t i = (t / inner) % n;
  const double* base = phi + (t - i * inner);
  auto P = [&](int64_t k) {
    int64_t r = (i + k) % n;
    if (r < 0) r += n;
    return base[r * inner];
  };
  double d;
  if (order == 2)
    d = (P(1) - P(-1)) / (2.0 * h);
  else if (order == 4)
    d = (8.0 * (P(1) - P(-1)) - (P(2) - P(-2))) / (12.0 * h);
  else
    d = (45.0 * (P(1) - P(-1)) - 9.0 * (P(2) - P(-2)) + (P(3) - P(-3))) / (60.0 * h);
  accel[t] = -d;
}

// ---- isolated boundaries (doubling-up method) -----------------------------
// the density in the low corner of the doubled grid, zero elsewhere
__global__ void iso_pad_kernel(const double* __restrict__ rho, double2* __restrict__ out, int3 n,
                               int3 m, int64_t ms) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ms;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(q % m.z);
    const int j = (int)((q / m.z) % m.y);
    const int i = (int)(q / ((int64_t)m.y * m.z));
    double v = 0.0;
    if (i < n.x && j < n.y && k < n.z) v = rho[((int64_t)i * n.y + j) * n.z + k];
    out[q] = make_double2(v, 0.0);
  }
}

__global__ void real_part_kernel(const double2* __restrict__ c, double* __restrict__ r, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    r[q] = c[q].x;
}

// potential of the physical cells and the FDA force from the doubled
// potential (its values beyond the physical cells are the isolated
// potential there); pd holds the unnormalised inverse DFT
__global__ void iso_force_kernel(const double2* __restrict__ pd, int3 n, int3 m, double scale,
                                 double3 h, int order, double* __restrict__ phi,
                                 double* __restrict__ accel, int64_t nxs) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nxs;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % n.z);
    const int j = (int)((t / n.z) % n.y);
    const int i = (int)(t / ((int64_t)n.y * n.z));
    const int64_t q = ((int64_t)i * m.y + j) * m.z + k;
    phi[t] = pd[q].x * scale;
    const int pos[3] = {i, j, k};
    const int mm[3] = {m.x, m.y, m.z};
    const int64_t inner[3] = {(int64_t)m.y * m.z, (int64_t)m.z, 1};
    const double hh[3] = {h.x, h.y, h.z};
    for (int l = 0; l < 3; ++l) {
      const double2* base = pd + (q - (int64_t)pos[l] * inner[l]);
      auto P = [&](int kk) {
        int r = (pos[l] + kk) % mm[l];
        if (r < 0) r += mm[l];
        return base[(int64_t)r * inner[l]].x * scale;
      };
      double d;
      if (order == 2)
        d = (P(1) - P(-1)) / (2.0 * hh[l]);
      else if (order == 4)
        d = (8.0 * (P(1) - P(-1)) - (P(2) - P(-2))) / (12.0 * hh[l]);
      else
        d = (45.0 * (P(1) - P(-1)) - 9.0 * (P(2) - P(-2)) + (P(3) - P(-3))) / (60.0 * hh[l]);
      accel[(int64_t)l * nxs + t] = -d;
    }
  }
}

// ---- initialisation and conversions -----------------------------------
template <typename T>
__global__ void init_separable_kernel(T* __restrict__ f, const double* __restrict__ s,
                                      const double* __restrict__ g1, const double* __restrict__ g2,
                                      const double* __restrict__ g3, int D, int64_t nv1,
                                      int64_t nv2, int64_t nv3, int64_t nvs, int64_t total) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ix = t / nvs;
    int64_t iv = t - ix * nvs;
    double v = s[ix];
    if (D == 1) {
      v = v * g1[iv];
    } else if (D == 2) {
      const int64_t j2 = iv % nv2, j1 = iv / nv2;
      v = v * g1[j1];
      v = v * g2[j2];
    } else {
      const int64_t j3 = iv % nv3;
      iv /= nv3;
      const int64_t j2 = iv % nv2, j1 = iv / nv2;
      v = v * g1[j1];
      v = v * g2[j2];
      v = v * g3[j3];
    }
    f[t] = (T)v;
  }
  (void)nv1;
}

template <typename T>
__global__ void from_double_kernel(T* __restrict__ f, const double* __restrict__ src, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    f[t] = (T)src[t];
}

template <typename T>
__global__ void to_double_kernel(const T* __restrict__ f, double* __restrict__ dst, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = (double)f[t];
}

// ---- diagnostics --------------------------------------------------------
// partials[b*4 + 0..3] = (sum, compensation, min, max) and
// partials[nblocks*4 + b] = count of non-finite values, per block b.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) diag_f_kernel(const T* __restrict__ f, int64_t n,
                                                    double* __restrict__ partials) {
  KSum acc{0.0, 0.0};
  double mn = INFINITY, mx = -INFINITY;
  double bad = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) {
    const double v = (double)f[t];
    if (!isfinite(v)) {
      bad += 1.0;
      continue;
    }
    kadd(acc, v);
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  KSum tot = block_ksum<NT>(acc);
  __shared__ double smn[NT], smx[NT], sbad[NT];
  smn[threadIdx.x] = mn;
  smx[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + off]);
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + off]);
      sbad[threadIdx.x] += sbad[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = tot.s;
    partials[blockIdx.x * 4 + 1] = tot.c;
    partials[blockIdx.x * 4 + 2] = smn[0];
    partials[blockIdx.x * 4 + 3] = smx[0];
    partials[(int64_t)gridDim.x * 4 + blockIdx.x] = sbad[0];
  }
}

// out[0] = sum |a|^2 over all components and cells; out[1], out[2] =
// real/imaginary part of sum_x a_1(x) exp(-2 pi i x1_index / nx1).
template <int NT>
__global__ void __launch_bounds__(NT) diag_field_kernel(const double* __restrict__ accel, int D,
                                                        int64_t nxs, int64_t nx1, int64_t inner1,
                                                        double* __restrict__ out) {
  KSum e{0.0, 0.0}, cr{0.0, 0.0}, ci{0.0, 0.0};
  for (int64_t t = threadIdx.x; t < (int64_t)D * nxs; t += NT) {
    const double a = accel[t];
    kadd(e, a * a);
  }
  for (int64_t t = threadIdx.x; t < nxs; t += NT) {
    const int64_t i1 = t / inner1;
    const double ang = -2.0 * M_PI * (double)(i1 % nx1) / (double)nx1;
    double sn, cs;
    sincos(ang, &sn, &cs);
    kadd(cr, accel[t] * cs);
    kadd(ci, accel[t] * sn);
  }
  KSum te = block_ksum<NT>(e);
  KSum tr = block_ksum<NT>(cr);
  KSum ti = block_ksum<NT>(ci);
  if (threadIdx.x == 0) {
    out[0] = te.s + te.c;
    out[1] = tr.s + tr.c;
    out[2] = ti.s + ti.c;
  }
}

// f <- cb * b + cf * f (the stage combinations of Eq. (RK)), grid-stride
__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }
inline unsigned grid_capped(int64_t n, int nt) {
  int64_t b = (n + nt - 1) / nt;
  return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

}  // namespace

hipError_t launch_moment(int dtype, const void* f, int64_t nxs, int64_t nvs, double dvol,
                         double* rho, hipStream_t s) {
  if (nxs <= 0) return hipSuccess;
  constexpr int NT = 256;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL((moment_kernel<double, NT>), dim3((unsigned)nxs), dim3(NT), 0, s,
                       (const double*)f, nvs, dvol, rho);
  else
    hipLaunchKernelGGL((moment_kernel<float, NT>), dim3((unsigned)nxs), dim3(NT), 0, s,
                       (const float*)f, nvs, dvol, rho);
  return hipGetLastError();
}

hipError_t launch_moment_reduce(const double* part, int n, int64_t ncol, int64_t nsub, double dvol,
                                double* rho, hipStream_t s) {
  const int64_t total = ncol * n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(moment_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     part, n, ncol, nsub, dvol, rho);
  return hipGetLastError();
}

hipError_t launch_poisson(const double* rho, double* phi, double* accel, double2* bufA,
                          double2* bufB, const double2* twiddles, const int64_t* tw_off,
                          const double* green, int D, const int64_t* nx, const double* h,
                          int order, hipStream_t s) {
  int64_t nxs = 1;
  for (int l = 0; l < D; ++l) nxs *= nx[l];
  constexpr int NT = 256;
  hipLaunchKernelGGL(real_to_complex_kernel, dim3(blocks_for(nxs, NT)), dim3(NT), 0, s, rho, bufA,
                     nxs);
  double2* cur = bufA;
  double2* oth = bufB;
  for (int pass = 0; pass < 2; ++pass) {
    for (int l = 0; l < D; ++l) {
      int64_t inner = 1;
      for (int k = l + 1; k < D; ++k) inner *= nx[k];
      hipLaunchKernelGGL(dft_axis_kernel, dim3(blocks_for(nxs, NT)), dim3(NT), 0, s, cur, oth,
                         nxs, nx[l], inner, twiddles + tw_off[l], pass);
      double2* t = cur;
      cur = oth;
      oth = t;
    }
    if (pass == 0)
      hipLaunchKernelGGL(green_kernel, dim3(blocks_for(nxs, NT)), dim3(NT), 0, s, cur, green, nxs);
  }
  hipLaunchKernelGGL(complex_to_real_kernel, dim3(blocks_for(nxs, NT)), dim3(NT), 0, s, cur, phi,
                     nxs, 1.0 / (double)nxs);
  for (int l = 0; l < D; ++l) {
    int64_t inner = 1;
    for (int k = l + 1; k < D; ++k) inner *= nx[k];
    hipLaunchKernelGGL(fda_kernel, dim3(blocks_for(nxs, NT)), dim3(NT), 0, s, phi,
                       accel + (int64_t)l * nxs, nxs, nx[l], inner, h[l], order);
  }
  return hipGetLastError();
}

// Three DFT passes over the doubled grid (sizes m, twiddles per axis at
// tw + tw_off[l]); returns the buffer holding the result.
static double2* dft3(double2* a, double2* b, const int64_t* m, const double2* tw,
                     const int64_t* tw_off, int conj, hipStream_t s) {
  const int64_t ms = m[0] * m[1] * m[2];
  constexpr int NT = 256;
  double2* cur = a;
  double2* oth = b;
  for (int l = 0; l < 3; ++l) {
    int64_t inner = 1;
    for (int k = l + 1; k < 3; ++k) inner *= m[k];
    hipLaunchKernelGGL(dft_axis_kernel, dim3(blocks_for(ms, NT)), dim3(NT), 0, s, cur, oth, ms,
                       m[l], inner, tw + tw_off[l], conj);
    double2* t = cur;
    cur = oth;
    oth = t;
  }
  return cur;
}

hipError_t launch_iso_green(double2* a, double2* b, const double2* tw, const int64_t* tw_off,
                            const int64_t* m, double* ghat, hipStream_t s) {
  const int64_t ms = m[0] * m[1] * m[2];
  double2* res = dft3(a, b, m, tw, tw_off, 0, s);
  hipLaunchKernelGGL(real_part_kernel, dim3(grid_capped(ms, 256)), dim3(256), 0, s, res, ghat, ms);
  return hipGetLastError();
}

hipError_t launch_poisson_isolated(const double* rho, double* phi, double* accel, double2* a,
                                   double2* b, const double2* tw, const int64_t* tw_off,
                                   const double* ghat, const int64_t* nx, const double* h,
                                   int order, hipStream_t s) {
  const int64_t m[3] = {2 * nx[0], 2 * nx[1], 2 * nx[2]};
  const int64_t ms = m[0] * m[1] * m[2], nxs = nx[0] * nx[1] * nx[2];
  const int3 n3 = make_int3((int)nx[0], (int)nx[1], (int)nx[2]);
  const int3 m3 = make_int3((int)m[0], (int)m[1], (int)m[2]);
  hipLaunchKernelGGL(iso_pad_kernel, dim3(grid_capped(ms, 256)), dim3(256), 0, s, rho, a, n3, m3,
                     ms);
  double2* fwd = dft3(a, b, m, tw, tw_off, 0, s);
  hipLaunchKernelGGL(green_kernel, dim3(blocks_for(ms, 256)), dim3(256), 0, s, fwd, ghat, ms);
  double2* other = fwd == a ? b : a;
  double2* inv = dft3(fwd, other, m, tw, tw_off, 1, s);
  hipLaunchKernelGGL(iso_force_kernel, dim3(grid_capped(nxs, 256)), dim3(256), 0, s, inv, n3, m3,
                     1.0 / (double)ms, make_double3(h[0], h[1], h[2]), order, phi, accel, nxs);
  return hipGetLastError();
}

hipError_t launch_init_separable(int dtype, void* f, const double* sx, const double* g1,
                                 const double* g2, const double* g3, int D, const int64_t* nv,
                                 int64_t nxs, int64_t nvs, hipStream_t st) {
  const int64_t total = nxs * nvs;
  constexpr int NT = 256;
  const unsigned grid = grid_capped(total, NT);
  const int64_t n1 = nv[0], n2 = D > 1 ? nv[1] : 1, n3 = D > 2 ? nv[2] : 1;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(init_separable_kernel<double>, dim3(grid), dim3(NT), 0, st, (double*)f, sx,
                       g1, g2, g3, D, n1, n2, n3, nvs, total);
  else
    hipLaunchKernelGGL(init_separable_kernel<float>, dim3(grid), dim3(NT), 0, st, (float*)f, sx,
                       g1, g2, g3, D, n1, n2, n3, nvs, total);
  return hipGetLastError();
}

hipError_t launch_from_double(int dtype, void* f, const double* src, int64_t n, hipStream_t s) {
  constexpr int NT = 256;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(from_double_kernel<double>, dim3(grid_capped(n, NT)), dim3(NT), 0, s,
                       (double*)f, src, n);
  else
    hipLaunchKernelGGL(from_double_kernel<float>, dim3(grid_capped(n, NT)), dim3(NT), 0, s,
                       (float*)f, src, n);
  return hipGetLastError();
}

hipError_t launch_to_double(int dtype, const void* f, double* dst, int64_t n, hipStream_t s) {
  constexpr int NT = 256;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(to_double_kernel<double>, dim3(grid_capped(n, NT)), dim3(NT), 0, s,
                       (const double*)f, dst, n);
  else
    hipLaunchKernelGGL(to_double_kernel<float>, dim3(grid_capped(n, NT)), dim3(NT), 0, s,
                       (const float*)f, dst, n);
  return hipGetLastError();
}

hipError_t launch_diag_f(int dtype, const void* f, int64_t n, double* partials, int nblocks,
                         hipStream_t s) {
  constexpr int NT = 256;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL((diag_f_kernel<double, NT>), dim3(nblocks), dim3(NT), 0, s,
                       (const double*)f, n, partials);
  else
    hipLaunchKernelGGL((diag_f_kernel<float, NT>), dim3(nblocks), dim3(NT), 0, s,
                       (const float*)f, n, partials);
  return hipGetLastError();
}

hipError_t launch_diag_field(const double* accel, int D, int64_t nxs, int64_t nx1, int64_t inner1,
                             double* out, hipStream_t s) {
  constexpr int NT = 256;
  hipLaunchKernelGGL((diag_field_kernel<NT>), dim3(1), dim3(NT), 0, s, accel, D, nxs, nx1, inner1,
                     out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  constexpr int NT = 256;
  const int64_t blocks = std::min<int64_t>((n + NT - 1) / NT, 256 * 64);
  if (n > 0)
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(NT), 0, s,
                       (const uint4*)src, (uint4*)dst, n);
  return hipGetLastError();
}

hipError_t launch_velocity_moments(int dtype, const void* f, int D, const int64_t* nv,
                                   const double* vlo, const double* dv, int64_t nxs,
                                   double* rho, double* mean, double* disp, hipStream_t s) {
  int64_t nvs = 1;
  double dvol = 1.0;
  for (int l = 0; l < D; ++l) {
    nvs *= nv[l];
    dvol *= dv[l];
  }
  const int3 n3 = make_int3((int)nv[0], D > 1 ? (int)nv[1] : 1, D > 2 ? (int)nv[2] : 1);
  const double3 lo3 = make_double3(vlo[0], D > 1 ? vlo[1] : 0.0, D > 2 ? vlo[2] : 0.0);
  const double3 dv3 = make_double3(dv[0], D > 1 ? dv[1] : 1.0, D > 2 ? dv[2] : 1.0);
  constexpr int NT = 256;
  if (D < 1 || D > 3) return hipErrorInvalidValue;
  auto go = [&](auto tag, auto axes) {
    using T = decltype(tag);
    hipLaunchKernelGGL((velocity_moments_kernel<T, NT, decltype(axes)::value>), dim3((unsigned)nxs),
                       dim3(NT), 0, s, (const T*)f, D, nvs, n3, lo3, dv3, dvol, nxs, rho, mean,
                       disp);
  };
  using A1 = std::integral_constant<int, 1>;
  using A2 = std::integral_constant<int, 2>;
  using A3 = std::integral_constant<int, 3>;
  if (dtype == SLMPP_F64) {
    if (D == 1) go(0.0, A1{});
    if (D == 2) go(0.0, A2{});
    if (D == 3) go(0.0, A3{});
  } else {
    if (D == 1) go(0.0f, A1{});
    if (D == 2) go(0.0f, A2{});
    if (D == 3) go(0.0f, A3{});
  }
  return hipGetLastError();
}

hipError_t launch_velocity_distribution(int dtype, const void* f, int64_t nxs, int64_t nvs,
                                        double xvol, double* F, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((nvs + 255) / 256, 4096);
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(velocity_distribution_kernel<double>, dim3((unsigned)blocks), dim3(256), 0,
                       s, (const double*)f, nxs, nvs, xvol, F);
  else
    hipLaunchKernelGGL(velocity_distribution_kernel<float>, dim3((unsigned)blocks), dim3(256), 0,
                       s, (const float*)f, nxs, nvs, xvol, F);
  return hipGetLastError();
}

}  // namespace slmpp
