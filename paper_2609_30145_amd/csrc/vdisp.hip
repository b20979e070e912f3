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
// parts of one complex FP64 transform held in LDS (real and imaginary parts in two arrays,
// one pad word every 16): a Stockham (self-sorting) transform in passes of radix 16 (then
// one of 8, 4 or 2 for the remaining factor), each thread reading its R values of a pass,
// twiddling them, transforming them in registers (16 = 4 x 4) and writing them back after
// a barrier; the product with both rows' Gaussians on conjugate frequency pairs
// (Z'_k = (H_a + H_b)/2 Z_k + (H_a - H_b)/2 conj(Z_{n-k}), which gives (x * h_a) + i (y * h_b)
// after the inverse since both H are real and even), stored conjugated, so that the same
// forward passes and a conjugation give the inverse.  Twiddles e^{-2 pi i k / n} come from
// the observation's table for k < n / 2 (FP64 cos and sin evaluated on the host; the other
// half is their negation).  A row with sigma_gal = 0 is left as it is; one outside
// [0, sigma_max] (NaN included) gets NaN over its whole row, hence a NaN model and logL.
#include "common.h"
#include "kernels.h"

namespace sps {

constexpr int kVdThreads = 256;

__device__ __forceinline__ int vd_pad(int i) { return i + (i >> 4); }

// e^{-2 pi i k / n} for 0 <= k < n from the half table
__device__ __forceinline__ void vd_twiddle(const double *__restrict__ tw, int k, int n, double &c, double &s) {
  const int h = n >> 1;
  const int kk = k < h ? k : k - h;
  c = tw[2 * kk];
  s = tw[2 * kk + 1];
  if (k >= h) {
    c = -c;
    s = -s;
  }
}

__device__ __forceinline__ void bfly4(double &r0, double &i0, double &r1, double &i1, double &r2, double &i2,
                                      double &r3, double &i3) {
  // X_k = sum_s a_s (-i)^{ks}, natural order in and out
  const double t0r = r0 + r2, t0i = i0 + i2, t1r = r0 - r2, t1i = i0 - i2;
  const double t2r = r1 + r3, t2i = i1 + i3, t3r = i1 - i3, t3i = r3 - r1;   // (a1 - a3)(-i)
  r0 = t0r + t2r;
  i0 = t0i + t2i;
  r2 = t0r - t2r;
  i2 = t0i - t2i;
  r1 = t1r + t3r;
  i1 = t1i + t3i;
  r3 = t1r - t3r;
  i3 = t1i - t3i;
}

__device__ __forceinline__ void cmul_c(double &r, double &i, double c, double s) {
  const double t = r * c - i * s;
  i = r * s + i * c;
  r = t;
}

// DFT of R values in registers, natural order in and out
template <int R>
__device__ __forceinline__ void dft_regs(double *vr, double *vi) {
  if constexpr (R == 2) {
    const double ar = vr[0], ai = vi[0];
    vr[0] = ar + vr[1];
    vi[0] = ai + vi[1];
    vr[1] = ar - vr[1];
    vi[1] = ai - vi[1];
  } else if constexpr (R == 4) {
    bfly4(vr[0], vi[0], vr[1], vi[1], vr[2], vi[2], vr[3], vi[3]);
  } else if constexpr (R == 8) {
    // 2 x 4: s = 2 s1 + s2, r = r1 + 4 r2
    bfly4(vr[0], vi[0], vr[2], vi[2], vr[4], vi[4], vr[6], vi[6]);
    bfly4(vr[1], vi[1], vr[3], vi[3], vr[5], vi[5], vr[7], vi[7]);
    constexpr double h = 0.70710678118654752440;   // e^{-2 pi i r1 / 8}, r1 = 1, 2, 3
    cmul_c(vr[3], vi[3], h, -h);
    cmul_c(vr[5], vi[5], 0.0, -1.0);
    cmul_c(vr[7], vi[7], -h, -h);
    double o[16];
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1) {
      const double ar = vr[2 * r1], ai = vi[2 * r1], br = vr[2 * r1 + 1], bi = vi[2 * r1 + 1];
      o[2 * r1] = ar + br;
      o[2 * r1 + 1] = ai + bi;
      o[8 + 2 * r1] = ar - br;
      o[8 + 2 * r1 + 1] = ai - bi;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      vr[r] = o[2 * r];
      vi[r] = o[2 * r + 1];
    }
  } else {
    static_assert(R == 16, "radix 2, 4, 8 or 16");
    // 4 x 4: s = 4 s1 + s2, r = r1 + 4 r2; inner transforms over s1, twiddles
    // e^{-2 pi i s2 r1 / 16}, outer transforms over s2
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
      bfly4(vr[s2], vi[s2], vr[4 + s2], vi[4 + s2], vr[8 + s2], vi[8 + s2], vr[12 + s2], vi[12 + s2]);
    // after the inner transforms, value (s2, r1) sits at 4 r1 + s2
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
    cmul_c(vr[4 + 1], vi[4 + 1], c1, -s1);    // s2 = 1, r1 = 1: k = 1
    cmul_c(vr[8 + 1], vi[8 + 1], h, -h);      // s2 = 1, r1 = 2: k = 2
    cmul_c(vr[12 + 1], vi[12 + 1], s1, -c1);  // s2 = 1, r1 = 3: k = 3
    cmul_c(vr[4 + 2], vi[4 + 2], h, -h);      // s2 = 2, r1 = 1: k = 2
    cmul_c(vr[8 + 2], vi[8 + 2], 0.0, -1.0);  // s2 = 2, r1 = 2: k = 4
    cmul_c(vr[12 + 2], vi[12 + 2], -h, -h);   // s2 = 2, r1 = 3: k = 6
    cmul_c(vr[4 + 3], vi[4 + 3], s1, -c1);    // s2 = 3, r1 = 1: k = 3
    cmul_c(vr[8 + 3], vi[8 + 3], -h, -h);     // s2 = 3, r1 = 2: k = 6
    cmul_c(vr[12 + 3], vi[12 + 3], -c1, s1);  // s2 = 3, r1 = 3: k = 9
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1)
      bfly4(vr[4 * r1], vi[4 * r1], vr[4 * r1 + 1], vi[4 * r1 + 1], vr[4 * r1 + 2], vi[4 * r1 + 2], vr[4 * r1 + 3],
            vi[4 * r1 + 3]);
    // value (r1, r2) now at 4 r1 + r2; output r = r1 + 4 r2
    double o[32];
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1)
#pragma unroll
      for (int r2 = 0; r2 < 4; ++r2) {
        o[2 * (r1 + 4 * r2)] = vr[4 * r1 + r2];
        o[2 * (r1 + 4 * r2) + 1] = vi[4 * r1 + r2];
      }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      vr[r] = o[2 * r];
      vi[r] = o[2 * r + 1];
    }
  }
}

// One Stockham pass of radix R over n = 2^lg values with sub-transform length Ns = 2^ls:
// item j reads x[j + r n/R], times e^{-2 pi i (j mod Ns) r / (Ns R)}, transforms, and
// writes x[(j div Ns) Ns R + (j mod Ns) + r Ns].  Every read precedes every write.
template <int R>
__device__ __forceinline__ void vd_pass(double *re, double *im, int n, int lg, int ls, const double *__restrict__ tw,
                                        int tid) {
  constexpr int lgR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  constexpr int J = kVdispMaxFFT / (R * kVdThreads);   // items per thread at the largest n
  const int nR = n >> lgR, Ns = 1 << ls, tsh = lg - ls - lgR;
  double vr[J][R], vi[J][R];
#pragma unroll
  for (int jj = 0; jj < J; ++jj) {
    const int j = tid + jj * kVdThreads;
    if (j < nR) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = vd_pad(j + r * nR);
        vr[jj][r] = re[q];
        vi[jj][r] = im[q];
      }
      const int jm = j & (Ns - 1);
      if (jm) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double c, s;
          vd_twiddle(tw, (jm * r) << tsh, n, c, s);
          cmul_c(vr[jj][r], vi[jj][r], c, s);
        }
      }
      dft_regs<R>(vr[jj], vi[jj]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < J; ++jj) {
    const int j = tid + jj * kVdThreads;
    if (j < nR) {
      const int base = ((j >> ls) << (ls + lgR)) + (j & (Ns - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = vd_pad(base + r * Ns);
        re[q] = vr[jj][r];
        im[q] = vi[jj][r];
      }
    }
  }
  __syncthreads();
}

// the whole forward transform: passes of 16, then one of the remaining radix
__device__ __forceinline__ void vd_fft(double *re, double *im, int n, int lg, const double *__restrict__ tw, int tid) {
  int ls = 0;
  while (lg - ls >= 4) {
    vd_pass<16>(re, im, n, lg, ls, tw, tid);
    ls += 4;
  }
  const int rem = lg - ls;
  if (rem == 3) vd_pass<8>(re, im, n, lg, ls, tw, tid);
  else if (rem == 2) vd_pass<4>(re, im, n, lg, ls, tw, tid);
  else if (rem == 1) vd_pass<2>(re, im, n, lg, ls, tw, tid);
}

template <typename T>
__global__ void __launch_bounds__(kVdThreads) k_vdisp(DevLib lib, VdispLaunch a) {
  extern __shared__ double vd_sm[];
  const int n = a.nfft, lg = a.log2n, tid = threadIdx.x;
  double *re = vd_sm, *im = vd_sm + vd_pad(n);
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

  // ---- F lambda^2 over the window, edge-padded, in natural order
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
    re[vd_pad(i)] = v[0];
    im[vd_pad(i)] = v[1];
  }
  __syncthreads();
  vd_fft(re, im, n, lg, tw, tid);

  // ---- both rows' Gaussians on the conjugate pairs (k, n - k), k = 0 .. n/2, stored
  // conjugated for the inverse
  {
    const double cn = kC_kms * dlnl * (double)n;
    const double ga = -2.0 * kPi * kPi * sg[0] * sg[0], gb = -2.0 * kPi * kPi * sg[1] * sg[1];
    for (int k = tid; k <= (n >> 1); k += kVdThreads) {
      const int m = (n - k) & (n - 1);
      const double nu = (double)k / cn, nu2 = nu * nu;
      const double Ha = act[0] ? exp(ga * nu2) : 1.0, Hb = act[1] ? exp(gb * nu2) : 1.0;
      const double P = 0.5 * (Ha + Hb), Q = 0.5 * (Ha - Hb);
      const int pk = vd_pad(k), pm = vd_pad(m);
      const double zr = re[pk], zi = im[pk], wr = re[pm], wi = im[pm];
      re[pk] = P * zr + Q * wr;
      im[pk] = -(P * zi - Q * wi);
      if (m != k) {
        re[pm] = P * wr + Q * zr;
        im[pm] = -(P * wi - Q * zi);
      }
    }
  }
  __syncthreads();
  vd_fft(re, im, n, lg, tw, tid);

  // ---- the window of F: conj(result) / n over lambda^2 (row a: real part, row b: imaginary)
  const double inv_n = 1.0 / (double)n;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!act[h]) continue;
    const double *buf = h ? im : re;
    const double sgn = h ? -inv_n : inv_n;
    for (int t = tid; t < nw[h]; t += kVdThreads) {
      const int k = j0[h] + t;
      Fr[h][k] = (T)(buf[vd_pad(t)] * sgn / lib.lam2_d[k]);
    }
  }
}

hipError_t launch_vdisp(const DevLib &lib, const VdispLaunch &vl, hipStream_t s) {
  if (vl.B_pad < 2 || (vl.B_pad & 1) || vl.nfft < 2 || vl.nfft > kVdispMaxFFT || (1 << vl.log2n) != vl.nfft)
    return hipErrorInvalidValue;
  const size_t sm = (size_t)(vl.nfft + (vl.nfft >> 4)) * 2 * sizeof(double);   // two padded arrays
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
