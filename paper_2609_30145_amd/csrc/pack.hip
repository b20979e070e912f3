// Load-time packing of the SSP library (done once per library).
//  * Q_ma: hydrogen-ionising photon rate of each unattenuated SSP (eq. C1), written
//    for f_lambda in Lsun/A: (Lsun/(h c)) * trapezoid of f lambda over lambda <= 912 A.
//  * the ionising continuum of nebular-covered ages is removed from their SSP rows (the
//    "combine" step of Fig. A1) when nebular emission is on; with an escape geometry it
//    has rows of its own, which the weight builder scales by f_ob (Sec. 2.3.2).
//  * young-first K order: young SSP rows, line-profile rows, ionising rows, old SSP rows.
//  * copies: FP64 and FP32 K-contiguous [N_pad][K_pad], FP32 N-contiguous [K_pad][N_pad]
//    for the adjoint, and 16-bit hi + residual planes with a per-row power of two.
#include <climits>

#include "common.h"
#include "kernels.h"

namespace sps {

__device__ __forceinline__ double src_value(const DevLib &lib, const PackLaunch &pk, int src, int n) {
  if (n >= lib.N || src == INT_MIN) return 0.0;
  if (src <= kIonSrc) {   // the raw ionising continuum of a nebular age (escape geometries)
    const int s = kIonSrc - src;
    return lib.wave_d[n] < kLamLyman ? pk.flux[(size_t)s * lib.N + n] : 0.0;
  }
  if (src < 0) return pk.lineprof[(size_t)(-1 - src) * lib.N + n];
  const int a = src % lib.n_age;
  if (pk.neb_mask && a >= lib.neb_a0 && a < lib.neb_a1 && lib.wave_d[n] < kLamLyman) return 0.0;
  return pk.flux[(size_t)src * lib.N + n];
}

__global__ void __launch_bounds__(256) k_rowstats(DevLib lib, PackLaunch pk) {
  __shared__ double red[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int src = pk.ksrc[k];
  double mx = 0.0, q = 0.0;
  for (int n = tid; n < lib.N; n += 256) {
    mx = fmax(mx, fabs(src_value(lib, pk, src, n)));
    if (src >= 0 && (src % lib.n_age) < lib.n_young && n + 1 < lib.N && lib.wave_d[n + 1] <= kLamLyman) {
      const double *f = pk.flux + (size_t)src * lib.N;
      q += 0.5 * (f[n] * lib.wave_d[n] + f[n + 1] * lib.wave_d[n + 1]) * (lib.wave_d[n + 1] - lib.wave_d[n]);
    }
  }
  red[tid] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double vmax = red[0];
  __syncthreads();
  red[tid] = q;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    pk.kexp[k] = vmax > 0.0 ? ilogb(vmax) - 14 : 0;
    pk.kexp16[k] = (int16_t)pk.kexp[k];   // |ilogb| of a double is below 1100
    if (src >= 0) {
      const int a = src % lib.n_age, zm = src / lib.n_age;
      if (a < lib.n_young) pk.Q[(size_t)zm * lib.n_young + a] = kLsun * kAng_cm * red[0] / (kHplanck * kC_cms);
    }
  }
}

__device__ __forceinline__ uint16_t pk_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t pk_f16(float f) {
  _Float16 h = (_Float16)f;
  return *reinterpret_cast<uint16_t *>(&h);
}

// 32 x 32 tiles: read along n, write K-contiguous copies through an LDS transpose.
__global__ void __launch_bounds__(256) k_pack(DevLib lib, PackLaunch pk) {
  __shared__ double tile[32][33];
  __shared__ int ke[32];
  const int n0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows of 32
  if (threadIdx.x < 32) ke[threadIdx.x] = pk.kexp[k0 + threadIdx.x];
  for (int kk = ty; kk < 32; kk += 8) {
    const int k = k0 + kk, n = n0 + tx;
    const double v = src_value(lib, pk, pk.ksrc[k], n);
    tile[kk][tx] = v;
    if (pk.L32n) pk.L32n[(size_t)k * lib.N_pad + n] = (float)v;
  }
  __syncthreads();
  for (int nn = ty; nn < 32; nn += 8) {
    const int n = n0 + nn, k = k0 + tx;
    const double v = tile[tx][nn];
    const size_t o = (size_t)n * lib.K_pad + k;
    if (pk.LT64) pk.LT64[o] = v;
    if (pk.LT32) pk.LT32[o] = (float)v;
    const double x = ldexp(v, -ke[tx]);
    if (pk.Hb) {
      const uint16_t h = pk_bf16((float)x);
      const float hf = __uint_as_float(((uint32_t)h) << 16);
      pk.Hb[o] = h;
      pk.Rb[o] = pk_bf16((float)(x - (double)hf));
    }
    if (pk.Hh) {
      const uint16_t h = pk_f16((float)x);
      _Float16 hv = *reinterpret_cast<const _Float16 *>(&h);
      pk.Hh[o] = h;
      pk.Rh[o] = pk_f16((float)(x - (double)(float)hv));
    }
  }
}

hipError_t launch_pack(const DevLib &lib, const PackLaunch &pk, hipStream_t s) {
  hipLaunchKernelGGL(k_rowstats, dim3(lib.K_pad), dim3(256), 0, s, lib, pk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pack, dim3(lib.N_pad / 32, lib.K_pad / 32), dim3(256), 0, s, lib, pk);
  return hipGetLastError();
}

}  // namespace sps
