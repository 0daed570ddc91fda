// Steps of the assimilation cycle around the analysis (Alg. 1): the perturbed
// observations of one assimilation time, and the squared error of the
// analysis mean that the RMSE of eq. (18) sums over assimilation times.
#include <mutex>

#include "device.h"

namespace enkfmc {

// Scratch of the allocation-free squared error: the partial sums of its first
// reduction level.  Each GPU holds its own copy until the process ends.  Host
// code never passes this name to a kernel (on the host it is a stand-in, not a
// device address); it uses the address that sq_error_scratch looked up.
static __device__ __align__(256) double scratch[kSqErrorParts];

namespace {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds; each multiplies words 0 and 2 by the two
// round multipliers, takes the 128-bit products apart and mixes their high
// halves with words 1, 3 and the round key.  The key is bumped by the two Weyl
// increments between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, x[0]), lo0 = kM0 * x[0];
    const uint64_t hi1 = __umul64hi(kM1, x[2]), lo1 = kM1 * x[2];
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
  }
}

// Uniform in (0, 1) from the top 52 bits: ((w >> 12) + 1/2) 2^-52, exact in
// double precision, never 0 or 1.
__device__ __forceinline__ double unit_open(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// Y^s[o][k] = y[o] + sqrt(r_o) xi(seed, cycle, o, k).  One thread per
// (observation o, group j of four members): the Philox block with key
// (seed, 0) and counter (j, o, cycle, 0) gives four uniforms u_0..u_3, and the
// Box-Muller transform turns (u_0, u_1) into members 4j, 4j+1 and (u_2, u_3)
// into 4j+2, 4j+3.
__global__ __launch_bounds__(256) void k_perturb(const double *__restrict__ y, const double *__restrict__ r_diag,
                                                 int64_t m, int N, uint64_t seed, uint64_t cycle,
                                                 double *__restrict__ Ys) {
  const int J = (N + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= m * J) return;
  const int64_t o = t / J;
  const int j = (int)(t % J);
  uint64_t x[4] = {(uint64_t)j, (uint64_t)o, cycle, 0};
  philox4x64_10(x, seed, 0);
  const double sd = sqrt(r_diag[o]), yo = y[o];
  double z[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double rho = sqrt(-2.0 * log(unit_open(x[2 * h])));
    double sn, cs;
    sincospi(2.0 * unit_open(x[2 * h + 1]), &sn, &cs);
    z[2 * h] = rho * cs;
    z[2 * h + 1] = rho * sn;
  }
  double *row = Ys + o * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (4 * j + i < N) row[4 * j + i] = yo + sd * z[i];
}

// Partial sums of (mean_k X_a[g][k] - x_ref[g])^2 over a fixed chunk of
// components per workgroup; the member sum runs k = 0..N-1 in order.
template <typename TX>
__global__ __launch_bounds__(256) void k_sq_error_parts(const TX *__restrict__ Xa, int64_t ld, int64_t n, int N,
                                                        const double *__restrict__ xref, int64_t chunk,
                                                        double *__restrict__ part) {
  __shared__ double red[4];
  const int64_t g0 = (int64_t)blockIdx.x * chunk;
  const int64_t g1 = g0 + chunk < n ? g0 + chunk : n;
  double s = 0.0;
  for (int64_t g = g0 + threadIdx.x; g < g1; g += 256) {
    const TX *row = Xa + g * ld;
    double a = 0.0;
    for (int k = 0; k < N; ++k) a += (double)row[k];
    const double e = a / (double)N - xref[g];
    s = fma(e, e, s);
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int nparts,
                                                   double *__restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

// eq. (18): out = sqrt(sum_t e_t / M) over the M squared errors, summed in a
// fixed order by one workgroup.
__global__ __launch_bounds__(256) void k_rmse(const double *__restrict__ sq, int64_t M, double *__restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < M; t += 256) s += sq[t];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[0] = sqrt(s / (double)M);
}

}  // namespace

hipError_t launch_rmse(const double *sq, int64_t M, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_rmse, dim3(1), dim3(256), 0, s, sq, M, out);
  return hipGetLastError();
}

hipError_t launch_perturb(const double *y, const double *r_diag, int64_t m, int N, uint64_t seed, uint64_t cycle,
                          double *Ys, hipStream_t s) {
  const int64_t threads = m * (int64_t)((N + 3) / 4);
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_perturb, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, y, r_diag, m, N, seed,
                     cycle, Ys);
  return hipGetLastError();
}

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current) and kept for later calls.
hipError_t sq_error_scratch(double **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (double *)ptr;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_sq_error(const void *Xa, int32_t dtype, int64_t ld, int64_t n, int N, const double *xref,
                           double *part, double *out, hipStream_t s) {
  const int64_t chunk = (n + kSqErrorParts - 1) / kSqErrorParts;
  if (dtype == ENKFMC_F32)
    hipLaunchKernelGGL(k_sq_error_parts<float>, dim3(kSqErrorParts), dim3(256), 0, s, (const float *)Xa, ld, n, N,
                       xref, chunk, part);
  else
    hipLaunchKernelGGL(k_sq_error_parts<double>, dim3(kSqErrorParts), dim3(256), 0, s, (const double *)Xa, ld, n,
                       N, xref, chunk, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double *)part, kSqErrorParts, out);
  return hipGetLastError();
}

}  // namespace enkfmc
