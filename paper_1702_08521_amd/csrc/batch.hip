// Field kernels of batched ensembles: the velocity moment over many runs in
// one launch, and the periodic Poisson solve + FDA force of each run by one
// workgroup working in LDS (Sec. 2.2, App. C).  Double precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "slmpp_internal.hpp"

namespace slmpp {
namespace {

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

// items[i] = (run, spatial cell); one wavefront per item.  Each lane sums
// its strided share of the velocity row (compensated), then the lanes are
// combined by a fixed shuffle tree, so the result does not depend on timing.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double vsum(mf4 v) {
  return ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
}
__device__ __forceinline__ double vsum(md2 v) { return v.x + v.y; }
template <typename T>
struct MVec {
  typedef mf4 type;
};
template <>
struct MVec<double> {
  typedef md2 type;
};

template <typename T>
__global__ void __launch_bounds__(256) batch_moment_kernel(const BatchRun* __restrict__ runs,
                                                           const int2* __restrict__ items,
                                                           int nitems) {
  using V = typename MVec<T>::type;
  constexpr int VN = 16 / sizeof(T);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int it = blockIdx.x * 4 + wave; it < nitems; it += gridDim.x * 4) {
    const int2 item = items[it];
    const BatchRun& r = runs[item.x];
    const T* b = reinterpret_cast<const T*>(r.f) + (int64_t)item.y * r.nvs;
    KSum acc{0.0, 0.0};
    constexpr int U = 4;
    if (r.nvs % VN == 0) {
      // 16-byte vectors; a vector's components are added in double first
      const V* bv = reinterpret_cast<const V*>(b);
      const int64_t nv = r.nvs / VN;
      int64_t k = lane;
      for (; k + (U - 1) * 64 < nv; k += U * 64) {
        V x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = __builtin_nontemporal_load(bv + k + u * 64);
#pragma unroll
        for (int u = 0; u < U; ++u) kadd(acc, vsum(x[u]));
      }
      for (; k < nv; k += 64) kadd(acc, vsum(bv[k]));
    } else {
      int64_t k = lane;
      for (; k + (U - 1) * 64 < r.nvs; k += U * 64) {
        T x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = b[k + u * 64];
#pragma unroll
        for (int u = 0; u < U; ++u) kadd(acc, (double)x[u]);
      }
      for (; k < r.nvs; k += 64) kadd(acc, (double)b[k]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double os = __shfl_down(acc.s, off, 64);
      const double oc = __shfl_down(acc.c, off, 64);
      kadd(acc, os);
      acc.c += oc;
    }
    if (lane == 0) r.rho[item.y] = r.dvol * (acc.s + acc.c);
  }
}

// rho of every listed run from the tile row sums its x_1 sweep left
// (grid.y = list entry): the row sums of one spatial cell added in tile
// order, compensated, in two interleaved accumulators.
__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchReduce* __restrict__ list) {
  const BatchReduce& b = list[blockIdx.y];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= b.ncol * b.n) return;
  const int64_t c = g / b.n;
  const int i = (int)(g - c * b.n);
  const double* p = b.part + c * b.nsub * b.n + i;
  KSum acc0{0.0, 0.0}, acc1{0.0, 0.0};
  int64_t q = 0;
  for (; q + 1 < b.nsub; q += 2) {
    const double x0 = p[q * b.n], x1 = p[(q + 1) * b.n];
    kadd(acc0, x0);
    kadd(acc1, x1);
  }
  if (q < b.nsub) kadd(acc0, p[q * b.n]);
  kadd(acc0, acc1.s);
  acc0.c += acc1.c;
  b.rho[(int64_t)i * b.ncol + c] = b.dvol * (acc0.s + acc0.c);
}

// Laplacian symbol times Delta^2 of the App. C stencils of order 2, 4, 6
__device__ __forceinline__ double lap_symbol(double th, int order) {
  const double a = sin(0.5 * th), b = sin(th), c = sin(1.5 * th);
  if (order == 2) return -4.0 * a * a;
  if (order == 4) return (b * b - 16.0 * a * a) / 3.0;
  return (-2.0 * c * c + 27.0 * b * b - 270.0 * a * a) / 45.0;
}

// In-LDS DFT of a D-dimensional complex array along axis l:
// out[.., k, ..] = sum_m in[.., m, ..] exp(sign 2 pi i m k / n), with the
// n roots of unity of the axis in tw (cos, sin of 2 pi q / n).  Sizes are
// at most kBatchMaxSpace, so 32-bit index arithmetic.
__device__ void lds_dft(const double2* in, double2* out, const double2* tw, int inner, int n,
                        int sign, int total) {
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int j = t % inner;
    const int k = (t / inner) % n;
    const int o = t / (inner * n);
    const double2* src = in + o * n * inner + j;
    // four interleaved partial sums (m mod 4): independent chains of LDS
    // reads and multiply-adds, added in a fixed order at the end
    double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
    int q = 0;
    int m = 0;
    for (; m + 3 < n; m += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double cs = tw[q].x;
        const double sn = sign * tw[q].y;
        const double2 x = src[(m + u) * inner];
        sr[u] += x.x * cs - x.y * sn;
        si[u] += x.x * sn + x.y * cs;
        q += k;
        if (q >= n) q -= n;
      }
    }
    for (; m < n; ++m) {
      const double cs = tw[q].x;
      const double sn = sign * tw[q].y;
      const double2 x = src[m * inner];
      sr[0] += x.x * cs - x.y * sn;
      si[0] += x.x * sn + x.y * cs;
      q += k;
      if (q >= n) q -= n;
    }
    out[t] = make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
  }
}

// One workgroup per run: rho -> phi_hat = G rho_hat -> phi -> accel.
// LDS: two complex work arrays, then per axis the roots of unity and the
// Laplacian symbol sym_l(k) / h_l^2 (see poisson_lds).  Up to one thread
// per spatial cell of the largest run (at most 1024): each DFT output is a
// serial chain of LDS reads, so the chains are spread over as many
// wavefronts as there are outputs.
__global__ void __launch_bounds__(1024) batch_poisson_kernel(const BatchRun* __restrict__ runs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BatchRun& r = runs[blockIdx.x];
  const int D = r.D;
  const int total = (int)r.nxs;
  // per-axis values in arrays indexed by constants only (the loops over
  // axes run to 3 with a guard and unroll), so that they stay in registers
  int nx[3] = {1, 1, 1}, inner[3] = {1, 1, 1}, toff[3] = {0, 0, 0};
  int ntw = 0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      nx[l] = (int)r.nx[l];
      toff[l] = ntw;
      ntw += nx[l];
    }
  }
#pragma unroll
  for (int l = 1; l >= 0; --l)
    if (l <= D - 2) inner[l] = inner[l + 1] * nx[l + 1];
  double2* A = reinterpret_cast<double2*>(smem);
  double2* B = A + total;
  double2* tw = B + total;  // roots of unity of axis l at tw + toff[l]
  double* sym = reinterpret_cast<double*>(tw + ntw);  // symbol of axis l at sym + toff[l]
  for (int t = threadIdx.x; t < ntw; t += blockDim.x) {
    int l = 0;
    if (1 < D && t >= toff[1]) l = 1;
    if (2 < D && t >= toff[2]) l = 2;
    const int k = t - (l == 0 ? toff[0] : (l == 1 ? toff[1] : toff[2]));
    const int n = l == 0 ? nx[0] : (l == 1 ? nx[1] : nx[2]);
    double sn, cs;
    sincospi(2.0 * (double)k / (double)n, &sn, &cs);
    tw[t] = make_double2(cs, sn);
    sym[t] = lap_symbol(2.0 * M_PI * (double)k / (double)n, r.poisson_order) / (r.h[l] * r.h[l]);
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) A[t] = make_double2(r.rho[t], 0.0);
  __syncthreads();
  double2* cur = A;
  double2* oth = B;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      lds_dft(cur, oth, tw + toff[l], inner[l], nx[l], -1, total);
      __syncthreads();
      double2* tmp = cur;
      cur = oth;
      oth = tmp;
    }
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    double L = 0.0;
    bool zero = true;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l < D) {
        const int k = (t / inner[l]) % nx[l];
        if (k) zero = false;
        L += sym[toff[l] + k];
      }
    }
    const double g = zero ? 0.0 : r.kappa / L;
    cur[t] = make_double2(cur[t].x * g, cur[t].y * g);
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      lds_dft(cur, oth, tw + toff[l], inner[l], nx[l], +1, total);
      __syncthreads();
      double2* tmp = cur;
      cur = oth;
      oth = tmp;
    }
  }
  // phi into the other buffer's real parts, then the force
  double* phi = reinterpret_cast<double*>(oth);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const double v = cur[t].x / (double)total;
    phi[t] = v;
    r.phi[t] = v;
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l >= D) break;
    const int n = nx[l], in = inner[l];
    const double h = r.h[l];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int i = (t / in) % n;
      const double* base = phi + (t - i * in);
      auto P = [&](int k) {
        int q = (i + k) % n;
        if (q < 0) q += n;
        return base[q * in];
      };
      double d;
      if (r.poisson_order == 2)
        d = (P(1) - P(-1)) / (2.0 * h);
      else if (r.poisson_order == 4)
        d = (8.0 * (P(1) - P(-1)) - (P(2) - P(-2))) / (12.0 * h);
      else
        d = (45.0 * (P(1) - P(-1)) - 9.0 * (P(2) - P(-2)) + (P(3) - P(-3))) / (60.0 * h);
      r.accel[(int64_t)l * total + t] = -d;
    }
  }
}

}  // namespace

hipError_t launch_batch_moment(int dtype, const BatchRun* runs, const int2* items, int nitems,
                               hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const int blocks = (nitems + 3) / 4;
  const int grid = blocks < 65536 ? blocks : 65536;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(batch_moment_kernel<double>, dim3(grid), dim3(256), 0, s, runs, items, nitems);
  else
    hipLaunchKernelGGL(batch_moment_kernel<float>, dim3(grid), dim3(256), 0, s, runs, items, nitems);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchReduce* list, int nlist, int64_t max_cells,
                               hipStream_t s) {
  if (nlist <= 0 || max_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_reduce_kernel, dim3((unsigned)((max_cells + 255) / 256), nlist), dim3(256),
                     0, s, list);
  return hipGetLastError();
}

hipError_t prepare_batch_sweep(int dtype, size_t lds_bytes);

namespace {
// two complex work arrays, plus a root of unity and a symbol value for
// every index of every axis (sum_l nx_l <= prod(nx) + 2 entries)
size_t poisson_lds(int max_nxs) {
  return sizeof(double2) * 2 * (size_t)max_nxs + (sizeof(double2) + sizeof(double)) * ((size_t)max_nxs + 2);
}
}  // namespace

hipError_t prepare_batch_kernels(int dtype, size_t sweep_lds, int max_nxs) {
  hipError_t e = prepare_batch_sweep(dtype, sweep_lds);
  const size_t lds = poisson_lds(max_nxs);
  if (e == hipSuccess && lds > 64 * 1024)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(batch_poisson_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e;
}

hipError_t launch_batch_poisson(const BatchRun* runs, int nruns, int max_nxs, hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  const size_t lds = poisson_lds(max_nxs);
  const int threads = std::min(1024, std::max(64, (max_nxs + 63) / 64 * 64));
  hipLaunchKernelGGL(batch_poisson_kernel, dim3(nruns), dim3(threads), lds, s, runs);
  return hipGetLastError();
}

}  // namespace slmpp
