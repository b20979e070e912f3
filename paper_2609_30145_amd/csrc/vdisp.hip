// Fourier stage of a free stellar velocity dispersion sigma_gal (Sec. 2.5 kinematics;
// App. F, the first of the continuum projection's two stages).
//
// Each point's rest-frame continuum F, over the window of nodes its projection reads
// (PointRow cov0 / cov_n, set by the weight builder), is turned into F lambda^2 (F_nu up to
// a per-point constant), written into a transform buffer of the observation's length n (a
// power of two) and padded with the window's last value for the larger half of the free
// length and its first value for the rest, multiplied in Fourier space by
// exp(-2 pi^2 sigma^2 nu^2), nu = k / (n c dln(lambda)) conjugate to c ln(lambda), and
// transformed back; the window of F is replaced by the result over lambda^2.  The
// observation's kernel (or its filters) and the IGM come after, in the projection.
//
// One workgroup per pair of sorted rows.  The two real windows are the real and imaginary
// parts of one complex FP64 transform held in LDS (2 n doubles): radix-2 decimation in
// time from bit-reversed loads, the product with both rows' Gaussians on conjugate
// frequency pairs (Z'_k = (H_a + H_b)/2 Z_k + (H_a - H_b)/2 conj(Z_{n-k}), which gives
// (x * h_a) + i (y * h_b) after the inverse since both H are real and even), then radix-2
// decimation in frequency with conjugate twiddles, read back in bit-reversed order.
// Twiddles e^{-2 pi i k / n}, k < n / 2, come from the observation's table (FP64 cos and
// sin evaluated on the host).  A row with sigma_gal = 0 is left as it is; one outside
// [0, sigma_max] (NaN included) gets NaN over its whole row, hence a NaN model and logL.
#include "common.h"
#include "kernels.h"

namespace sps {

constexpr int kVdThreads = 256;

__device__ __forceinline__ int bit_reverse(int i, int lg) { return (int)(__brev((unsigned)i) >> (32 - lg)); }

template <typename T>
__global__ void __launch_bounds__(kVdThreads) k_vdisp(DevLib lib, VdispLaunch a) {
  extern __shared__ double vd_sm[];
  const int n = a.nfft, lg = a.log2n, tid = threadIdx.x;
  double *re = vd_sm, *im = vd_sm + n;
  const DevObs *ob = a.obs;
  const double *__restrict__ tw = ob->vd_tw;
  const double dlnl = ob->vd_dlnl;
  int j0[2], nw[2];
  double sg[2];
  bool act[2];
  T *Fr[2];
  bool any = false;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = 2 * blockIdx.x + h;
    const PointRow &pr = a.rows[r];
    Fr[h] = (T *)a.F + (size_t)r * lib.N_pad;
    act[h] = false;
    j0[h] = 0;
    nw[h] = 0;
    sg[h] = 0.0;
    if (pr.b < 0) continue;
    const double s = a.theta[(size_t)pr.b * lib.P + lib.th_sgal];
    if (!(s >= 0.0 && s <= lib.vd_max)) {
      for (int k = tid; k < lib.N_pad; k += kVdThreads) Fr[h][k] = (T)__builtin_nan("");
      continue;
    }
    if (s == 0.0 || pr.cov_n <= 0) continue;
    act[h] = true;
    j0[h] = pr.cov0;
    nw[h] = min(pr.cov_n, n);   // the host sizes n to hold every window
    sg[h] = s;
    any = true;
  }
  if (!any) return;   // the same for every thread of the block

  // ---- load F lambda^2 over the window, edge-padded, at bit-reversed positions
  for (int i = tid; i < n; i += kVdThreads) {
    double v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v[h] = 0.0;
      if (act[h]) {
        const int m = nw[h], hp = (n - m + 1) >> 1;
        const int k = j0[h] + (i < m ? i : (i < m + hp ? m - 1 : 0));
        v[h] = (double)Fr[h][k] * lib.lam2_d[k];
      }
    }
    const int p = bit_reverse(i, lg);
    re[p] = v[0];
    im[p] = v[1];
  }
  __syncthreads();

  // ---- forward transform: decimation in time, natural order out
  for (int s = 0; s < lg; ++s) {
    const int half = 1 << s, tsh = lg - 1 - s;
    for (int q = tid; q < (n >> 1); q += kVdThreads) {
      const int pos = q & (half - 1);
      const int i0 = ((q >> s) << (s + 1)) + pos, i1 = i0 + half;
      const double wr = tw[2 * (pos << tsh)], wi = tw[2 * (pos << tsh) + 1];
      const double xr = re[i1], xi = im[i1], ar = re[i0], ai = im[i0];
      const double tr = wr * xr - wi * xi, ti = wr * xi + wi * xr;
      re[i0] = ar + tr;
      im[i0] = ai + ti;
      re[i1] = ar - tr;
      im[i1] = ai - ti;
    }
    __syncthreads();
  }

  // ---- both rows' Gaussians on the conjugate pairs (k, n - k), k = 0 .. n/2
  {
    const double cn = kC_kms * dlnl * (double)n;
    const double ga = -2.0 * kPi * kPi * sg[0] * sg[0], gb = -2.0 * kPi * kPi * sg[1] * sg[1];
    for (int k = tid; k <= (n >> 1); k += kVdThreads) {
      const int m = (n - k) & (n - 1);
      const double nu = (double)k / cn, nu2 = nu * nu;
      const double Ha = act[0] ? exp(ga * nu2) : 1.0, Hb = act[1] ? exp(gb * nu2) : 1.0;
      const double P = 0.5 * (Ha + Hb), Q = 0.5 * (Ha - Hb);
      const double zr = re[k], zi = im[k], wr = re[m], wi = im[m];
      re[k] = P * zr + Q * wr;
      im[k] = P * zi - Q * wi;
      if (m != k) {
        re[m] = P * wr + Q * zr;
        im[m] = P * wi - Q * zi;
      }
    }
  }
  __syncthreads();

  // ---- inverse transform: decimation in frequency, conjugate twiddles, bit-reversed out
  for (int s = lg - 1; s >= 0; --s) {
    const int half = 1 << s, tsh = lg - 1 - s;
    for (int q = tid; q < (n >> 1); q += kVdThreads) {
      const int pos = q & (half - 1);
      const int i0 = ((q >> s) << (s + 1)) + pos, i1 = i0 + half;
      const double wr = tw[2 * (pos << tsh)], wi = -tw[2 * (pos << tsh) + 1];
      const double ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
      re[i0] = ar + br;
      im[i0] = ai + bi;
      const double dr = ar - br, di = ai - bi;
      re[i1] = dr * wr - di * wi;
      im[i1] = dr * wi + di * wr;
    }
    __syncthreads();
  }

  // ---- the window of F: the result over n lambda^2
  const double inv_n = 1.0 / (double)n;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!act[h]) continue;
    const double *buf = h ? im : re;
    for (int t = tid; t < nw[h]; t += kVdThreads) {
      const int k = j0[h] + t;
      Fr[h][k] = (T)(buf[bit_reverse(t, lg)] * inv_n / lib.lam2_d[k]);
    }
  }
}

hipError_t launch_vdisp(const DevLib &lib, const VdispLaunch &vl, hipStream_t s) {
  if (vl.B_pad < 2 || (vl.B_pad & 1) || vl.nfft < 2 || vl.nfft > kVdispMaxFFT || (1 << vl.log2n) != vl.nfft)
    return hipErrorInvalidValue;
  const size_t sm = (size_t)vl.nfft * 2 * sizeof(double);
  const void *fn = vl.f64 ? (const void *)k_vdisp<double> : (const void *)k_vdisp<float>;
  if (sm > 65536) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
  }
  if (vl.f64)
    hipLaunchKernelGGL(k_vdisp<double>, dim3(vl.B_pad / 2), dim3(kVdThreads), sm, s, lib, vl);
  else
    hipLaunchKernelGGL(k_vdisp<float>, dim3(vl.B_pad / 2), dim3(kVdThreads), sm, s, lib, vl);
  return hipGetLastError();
}

}  // namespace sps
