// Field kernels of batched ensembles: the velocity moment over many runs in
// one launch, and the periodic Poisson solve + FDA force of each run by one
// workgroup working in LDS (Sec. 2.2, App. C).  Double precision.
#include <hip/hip_runtime.h>

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

// items[i] = (run, spatial cell); one workgroup per item, fixed order.
template <typename T>
__global__ void __launch_bounds__(256) batch_moment_kernel(const BatchRun* __restrict__ runs,
                                                           const int2* __restrict__ items,
                                                           int nitems) {
  __shared__ double ss[256], sc[256];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BatchRun& r = runs[item.x];
    const T* b = reinterpret_cast<const T*>(r.f) + (int64_t)item.y * r.nvs;
    KSum acc{0.0, 0.0};
    for (int64_t k = threadIdx.x; k < r.nvs; k += 256) kadd(acc, (double)b[k]);
    ss[threadIdx.x] = acc.s;
    sc[threadIdx.x] = acc.c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        KSum a{ss[threadIdx.x], sc[threadIdx.x]};
        kadd(a, ss[threadIdx.x + off]);
        a.c += sc[threadIdx.x + off];
        ss[threadIdx.x] = a.s;
        sc[threadIdx.x] = a.c;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) r.rho[item.y] = r.dvol * (ss[0] + sc[0]);
    __syncthreads();
  }
}

// Laplacian symbol times Delta^2 of the App. C stencils of order 2, 4, 6
__device__ __forceinline__ double lap_symbol(double th, int order) {
  const double a = sin(0.5 * th), b = sin(th), c = sin(1.5 * th);
  if (order == 2) return -4.0 * a * a;
  if (order == 4) return (b * b - 16.0 * a * a) / 3.0;
  return (-2.0 * c * c + 27.0 * b * b - 270.0 * a * a) / 45.0;
}

// In-LDS DFT of a D-dimensional complex array along axis l:
// out[.., k, ..] = sum_m in[.., m, ..] exp(sign 2 pi i m k / n)
__device__ void lds_dft(const double2* in, double2* out, int D, const int64_t* nx, int l,
                        int sign, int total) {
  int64_t inner = 1;
  for (int k = l + 1; k < D; ++k) inner *= nx[k];
  const int n = (int)nx[l];
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int j = (int)(t % inner);
    const int k = (int)((t / inner) % n);
    const int o = (int)(t / (inner * n));
    const double2* src = in + (int64_t)o * n * inner + j;
    double sr = 0.0, si = 0.0;
    int q = 0;
    for (int m = 0; m < n; ++m) {
      double sn, cs;
      sincospi(2.0 * (double)q / (double)n, &sn, &cs);
      sn *= sign;
      const double2 x = src[(int64_t)m * inner];
      sr += x.x * cs - x.y * sn;
      si += x.x * sn + x.y * cs;
      q += k;
      if (q >= n) q -= n;
    }
    out[t] = make_double2(sr, si);
  }
}

// One workgroup per run: rho -> phi_hat = G rho_hat -> phi -> accel.
__global__ void __launch_bounds__(256) batch_poisson_kernel(const BatchRun* __restrict__ runs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BatchRun& r = runs[blockIdx.x];
  const int D = r.D;
  const int total = (int)r.nxs;
  double2* A = reinterpret_cast<double2*>(smem);
  double2* B = A + total;
  for (int t = threadIdx.x; t < total; t += blockDim.x) A[t] = make_double2(r.rho[t], 0.0);
  __syncthreads();
  double2* cur = A;
  double2* oth = B;
  for (int l = 0; l < D; ++l) {
    lds_dft(cur, oth, D, r.nx, l, -1, total);
    __syncthreads();
    double2* tmp = cur;
    cur = oth;
    oth = tmp;
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int64_t rem = t;
    double L = 0.0;
    bool zero = true;
    for (int l = D - 1; l >= 0; --l) {
      const int64_t k = rem % r.nx[l];
      rem /= r.nx[l];
      if (k) zero = false;
      const double th = 2.0 * M_PI * (double)k / (double)r.nx[l];
      L += lap_symbol(th, r.poisson_order) / (r.h[l] * r.h[l]);
    }
    const double g = zero ? 0.0 : r.kappa / L;
    cur[t] = make_double2(cur[t].x * g, cur[t].y * g);
  }
  __syncthreads();
  for (int l = 0; l < D; ++l) {
    lds_dft(cur, oth, D, r.nx, l, +1, total);
    __syncthreads();
    double2* tmp = cur;
    cur = oth;
    oth = tmp;
  }
  // phi into the other buffer's real parts, then the force
  double* phi = reinterpret_cast<double*>(oth);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const double v = cur[t].x / (double)total;
    phi[t] = v;
    r.phi[t] = v;
  }
  __syncthreads();
  for (int l = 0; l < D; ++l) {
    int64_t inner = 1;
    for (int k = l + 1; k < D; ++k) inner *= r.nx[k];
    const int64_t n = r.nx[l];
    const double h = r.h[l];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int64_t i = (t / inner) % n;
      const double* base = phi + (t - i * inner);
      auto P = [&](int64_t k) {
        int64_t q = (i + k) % n;
        if (q < 0) q += n;
        return base[q * inner];
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
  const int grid = nitems < 65536 ? nitems : 65536;
  if (dtype == SLMPP_F64)
    hipLaunchKernelGGL(batch_moment_kernel<double>, dim3(grid), dim3(256), 0, s, runs, items, nitems);
  else
    hipLaunchKernelGGL(batch_moment_kernel<float>, dim3(grid), dim3(256), 0, s, runs, items, nitems);
  return hipGetLastError();
}

hipError_t prepare_batch_sweep(int dtype, size_t lds_bytes);

hipError_t prepare_batch_kernels(int dtype, size_t sweep_lds, int max_nxs) {
  hipError_t e = prepare_batch_sweep(dtype, sweep_lds);
  const size_t lds = 2 * sizeof(double2) * (size_t)max_nxs;
  if (e == hipSuccess && lds > 64 * 1024)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(batch_poisson_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e;
}

hipError_t launch_batch_poisson(const BatchRun* runs, int nruns, int max_nxs, hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  const size_t lds = 2 * sizeof(double2) * (size_t)max_nxs;
  hipLaunchKernelGGL(batch_poisson_kernel, dim3(nruns), dim3(256), lds, s, runs);
  return hipGetLastError();
}

}  // namespace slmpp
