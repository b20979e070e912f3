// Reverse pass of the forward model: d logL / d theta (exact gradient, FP64 output).
//
//   k_adj_proj   d logL / d F on the rest-frame grid from the photometric or spectral
//                projection (deterministic gathers), the direct redshift, logmass and
//                line terms, then the attenuation adjoint: G_Y = gF T_d T_BC,
//                G_O = gF T_d and the four dust-parameter sums (eq. D2).
//   k_bwd_*      dW = [G_Y | G_O] L^T, the transpose contraction (MFMA for FP32).
//   k_adj_prep   line luminosities (eq. C2) and SSP weights (App. B) back to theta,
//                including the SFH edges' dependence on t_univ(z).
#include <climits>

#include "kernels.h"
#include "runtime.h"

namespace sps {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// slots of the per-point adjoint scratch gbuf[r][16]
enum { GB_Z = 0, GB_TAU_BC, GB_ALPHA_BC, GB_TAU_DIFF, GB_DELTA, GB_LOGMASS, GB_N };

struct AdjArgs {
  const double *theta;
  int P, B, N_pad, n_line;
  const PointRow *rows;
  const DevObs *obs_table;
  const void *F, *Yatt;
  const double *gvec, *model;   // [B_pad][ld_g] (sorted rows)
  int ld_g;
  const double *Lline;          // [B_pad][n_line]
  double *scr;                  // [B_pad][ld_scr] per-node / per-pixel scratch
  int ld_scr;
  void *GY, *GO;                // [B_pad][N_pad]
  double *gbuf;                 // [B_pad][16]
  double *dLl;                  // [B_pad][n_line]
};

__device__ __forceinline__ double block_sum256(double v, double *red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double sigma_inst_at(const DevObs &ob, double lam, double *dsig_dlam) {
  // eq. F2 and its derivative in the observed wavelength
  double v = ob.lsf_value, dv = 0.0;
  if (ob.has_curve) {
    const int np = ob.n_data;
    if (lam <= ob.pix[0]) v = ob.lsf_vals[0];
    else if (lam >= ob.pix[np - 1]) v = ob.lsf_vals[np - 1];
    else {
      const int k = bracket(ob.pix, np, lam);
      dv = (ob.lsf_vals[k + 1] - ob.lsf_vals[k]) / (ob.pix[k + 1] - ob.pix[k]);
      v = ob.lsf_vals[k] + dv * (lam - ob.pix[k]);
    }
  }
  const double f = 2.3548200450309493, c = kC_kms;
  double s, ds;
  switch (ob.lsf_mode) {
    case 0: s = c / (f * v); ds = -c * dv / (f * v * v); break;
    case 1: s = c / v; ds = -c * dv / (v * v); break;
    case 2: s = c * v / (f * lam); ds = c / f * (dv / lam - v / (lam * lam)); break;
    case 3: s = c * v / lam; ds = c * (dv / lam - v / (lam * lam)); break;
    case 4: s = v; ds = dv; break;
    default: s = v / f; ds = dv / f; break;
  }
  *dsig_dlam = ds;
  return s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_proj(DevLib lib, AdjArgs a) {
  extern __shared__ double gFl[];     // [N] d logL / d F on the rest grid
  __shared__ double red[256];
  __shared__ double s_lnl[512], s_sl[512], s_dsl[512], s_F[512], s_T[512];
  const int r = blockIdx.x, tid = threadIdx.x;
  const PointRow pr = a.rows[r];
  if (pr.b < 0) return;
  const DevObs ob = a.obs_table[pr.obs];
  const int N = lib.N;
  const T *Fr = (const T *)a.F + (size_t)r * a.N_pad;
  const T *Yr = (const T *)a.Yatt + (size_t)r * a.N_pad;
  const double *gm = a.gvec + (size_t)r * a.ld_g;
  const double *mm = a.model + (size_t)r * a.ld_g;
  double *scr = a.scr + (size_t)r * a.ld_scr;
  const double z = pr.z, opz = 1.0 + z;
  const double Ez = sqrt(lib.Om * opz * opz * opz + 1.0 - lib.Om);
  const double ddl = pr.dc + opz * (kC_kms / lib.H0) * kMpc_cm / Ez;   // dD_L/dz [cm]
  const int chunk = (N + 255) / 256;
  const int n0 = min(tid * chunk, N), n1 = min(n0 + chunk, N);
  for (int n = n0; n < n1; ++n) gFl[n] = 0.0;
  double gz = 0.0, glm = 0.0, gtb = 0.0, gab = 0.0, gtd = 0.0, gdl = 0.0;
  for (int i = tid; i < ob.n_data; i += 256) glm += gm[i] * mm[i];

  if (ob.kind == 0) {
    // ---------------- photometry: m_b = A sum_j c_j interp(F)(lambda_j / (1+z))
    const double A = kC_cms * pr.scale_fnu / (opz * opz * kAng_cm * kAng_cm);
    const double dlnA = -1.0 / opz - 2.0 * ddl / pr.dl;
    for (int b = 0; b < ob.n_band; ++b) {
      const int j0 = ob.band_off[b], j1 = ob.band_off[b + 1];
      if (tid == 0) gz += gm[b] * dlnA * mm[b];
      for (int j = j0 + tid; j < j1; j += 256) {
        const double lr = ob.fw[j] / opz;
        double kk, t = 0.0, coef = gm[b] * A * ob.fr_d[j];
        if (lr < lib.wave_d[0]) kk = -2.0;
        else if (lr > lib.wave_d[N - 1]) kk = (double)(N + 1);
        else {
          const int k = wave_bracket(lib, lr);
          const double dw = lib.wave_d[k + 1] - lib.wave_d[k];
          t = (lr - lib.wave_d[k]) / dw;
          kk = (double)k;
          const double slope = ((double)Fr[k + 1] - (double)Fr[k]) / dw;
          gz += coef * slope * (-ob.fw[j] / (opz * opz));
        }
        scr[3 * j] = kk;
        scr[3 * j + 1] = t;
        scr[3 * j + 2] = coef;
      }
    }
    __syncthreads();
    // gather: each thread owns model pixels [n0, n1); bands and nodes in a fixed order
    if (n0 < n1) {
      for (int b = 0; b < ob.n_band; ++b) {
        const int j0 = ob.band_off[b], j1 = ob.band_off[b + 1];
        int lo = j0, hi = j1;   // first node with k >= n0 - 1
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (scr[3 * mid] < (double)(n0 - 1)) lo = mid + 1; else hi = mid;
        }
        for (int j = lo; j < j1; ++j) {
          const double kk = scr[3 * j];
          if (kk >= (double)n1) break;
          const int k = (int)kk;
          const double t = scr[3 * j + 1], coef = scr[3 * j + 2];
          if (k >= n0 && k < n1) gFl[k] += coef * (1.0 - t);
          if (k + 1 >= n0 && k + 1 < n1) gFl[k + 1] += coef * t;
        }
      }
    }
  } else {
    // ---------------- spectrum: m_i = (S sum_j w_ij F_j lambda_j^2 + lines_i) / f_AB
    const double S = pr.scale_fnu;
    const double dlnS = 1.0 / opz - 2.0 * ddl / pr.dl;
    const double lnopz = log1p(z);
    const int np = ob.n_data;
    const double lnw0 = lib.lnwave_d[0], lnw1 = lib.lnwave_d[N - 1];
    // per pixel: x, s (or -1 for a linear row), j0, j1, coefficient; stride 6
    for (int i = tid; i < np; i += 256) {
      const double gc = gm[i] / kFnuAB;
      const double x = ob.lnpix[i] - lnopz;
      double *q = scr + 6 * i;
      if (x < lnw0 || x > lnw1) {
        q[0] = x; q[1] = 0.0; q[2] = (double)INT_MAX; q[3] = -1.0; q[4] = 0.0;
        continue;
      }
      const double s = ob.ksig[i];
      const int k = lnwave_bracket(lib, x);
      const double dk = lib.lnwave_d[k + 1] - lib.lnwave_d[k];
      if (s < 0.5 * dk) {
        const double t = (x - lib.lnwave_d[k]) / dk;
        const double fk = (double)Fr[k] * lib.lam2_d[k], fk1 = (double)Fr[k + 1] * lib.lam2_d[k + 1];
        const double cont = fk + t * (fk1 - fk);
        gz += gc * (dlnS * S * cont + S * (fk1 - fk) * (-1.0 / (opz * dk)));
        q[0] = x; q[1] = -1.0; q[2] = (double)k; q[3] = (double)(k + 1); q[4] = gc * S; q[5] = t;
      } else {
        const int j0 = lnwave_lower_bound(lib, x - 5.0 * s);
        double G = 0.0, num = 0.0, dg = 0.0, dgf = 0.0;
        int j = j0;
        const double inv = 1.0 / s;
        for (; j < N; ++j) {
          const double u = (lib.lnwave_d[j] - x) * inv;
          if (u > 5.0) break;
          const double g = exp(-0.5 * u * u);
          const double fj = (double)Fr[j] * lib.lam2_d[j];
          G += g;
          num += g * fj;
          const double d = -u * g * inv / opz;
          dg += d;
          dgf += d * fj;
        }
        const double cont = num / G;
        gz += gc * (dlnS * S * cont + S * (dgf - cont * dg) / G);
        q[0] = x; q[1] = s; q[2] = (double)j0; q[3] = (double)(j - 1); q[4] = gc * S / G; q[5] = 0.0;
      }
    }
    // analytic lines on the pixels (eq. F6)
    const int nl = a.n_line;
    if (nl > 0) {
      const double Kf = pr.mass10 / (4.0 * kPi * pr.dl * pr.dl);
      const double Eb = 0.85 - 1.9 * pr.delta;
      for (int l = tid; l < nl; l += 256) {
        const double lw = lib.line_wave[l];
        const double lnlv = log(lw / kLamV);
        const double p = exp(pr.alpha_bc * lnlv), qd = exp(pr.delta * lnlv);
        const double Tl = exp(-pr.tau_bc * p - pr.tau_diff * qd * (lib.line_a[l] + Eb * lib.line_d[l]));
        const double lobs = opz * lw;
        double dsig;
        const double si = sigma_inst_at(ob, lobs, &dsig);
        const double sl = sqrt(ob.sigma_gas_kms * ob.sigma_gas_kms + si * si) / kC_kms;
        s_lnl[l] = log(lobs);
        s_sl[l] = sl;
        s_dsl[l] = si * dsig * lw / (kC_kms * kC_kms * sl);
        s_F[l] = a.Lline[(size_t)r * nl + l] * Tl * Kf;
        s_T[l] = Tl * Kf;
      }
      __syncthreads();
      // per line: gather over the pixels within kLineCut sigma (pixels sorted)
      for (int l = tid; l < nl; l += 256) {
        const double mu = s_lnl[l], sl = s_sl[l];
        int i = lower_bound_dev(ob.lnpix, np, mu - 10.0 * sl);
        double gFlx = 0.0, gzl = 0.0;
        for (; i < np && ob.lnpix[i] <= mu + 10.0 * sl; ++i) {
          const double u = (ob.lnpix[i] - mu) / sl;
          const double Nn = exp(-0.5 * u * u) / (2.5066282746310002 * sl);
          const double glp = gm[i] / kFnuAB * ob.pix[i] * kAng_cm / kC_cms;
          gFlx += glp * Nn;
          gzl += glp * s_F[l] * (Nn * u / sl / opz + Nn * (u * u - 1.0) / sl * s_dsl[l]);
        }
        gz += gzl + gFlx * s_F[l] * (-2.0 * ddl / pr.dl);
        a.dLl[(size_t)r * nl + l] = gFlx * s_T[l];
        const double lw = lib.line_wave[l];
        const double lnlv = log(lw / kLamV);
        const double p = exp(pr.alpha_bc * lnlv), qd = exp(pr.delta * lnlv);
        const double sh = lib.line_a[l] + Eb * lib.line_d[l];
        const double gf = gFlx * s_F[l];
        gtb += gf * (-p);
        gab += gf * (-pr.tau_bc * p * lnlv);
        gtd += gf * (-qd * sh);
        gdl += gf * (-pr.tau_diff * (qd * lnlv * sh - 1.9 * qd * lib.line_d[l]));
      }
    }
    __syncthreads();
    // prefix max of j1 (slot 3) and suffix min of j0 (slot 2): two-level scans
    {
      const int pc = (np + 255) / 256;
      const int i0 = min(tid * pc, np), i1 = min(i0 + pc, np);
      double mx = -1.0;
      for (int i = i0; i < i1; ++i) mx = fmax(mx, scr[6 * i + 3]);
      red[tid] = mx;
      __syncthreads();
      if (tid == 0)
        for (int q = 1; q < 256; ++q) red[q] = fmax(red[q], red[q - 1]);
      __syncthreads();
      double run = tid > 0 ? red[tid - 1] : -1.0;
      __syncthreads();
      for (int i = i0; i < i1; ++i) {
        run = fmax(run, scr[6 * i + 3]);
        scr[6 * np + i] = run;          // prefix max of j1
      }
      double mn = (double)INT_MAX;
      for (int i = i0; i < i1; ++i) mn = fmin(mn, scr[6 * i + 2]);
      red[tid] = mn;
      __syncthreads();
      if (tid == 0)
        for (int q = 254; q >= 0; --q) red[q] = fmin(red[q], red[q + 1]);
      __syncthreads();
      double run2 = tid < 255 ? red[tid + 1] : (double)INT_MAX;
      for (int i = i1 - 1; i >= i0; --i) {
        run2 = fmin(run2, scr[6 * i + 2]);
        scr[7 * np + i] = run2;         // suffix min of j0
      }
    }
    __syncthreads();
    if (n0 < n1) {
      int lo = 0, hi = np;   // first pixel whose prefix-max j1 reaches n0
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (scr[6 * np + mid] < (double)n0) lo = mid + 1; else hi = mid;
      }
      for (int i = lo; i < np && scr[7 * np + i] < (double)n1; ++i) {
        const double *q = scr + 6 * i;
        const int j0 = (int)fmax(q[2], (double)n0);
        const int j1 = (int)fmin(q[3], (double)(n1 - 1));
        if (j0 > j1) continue;
        if (q[1] < 0.0) {   // linear row
          const int k = (int)q[2];
          if (k >= n0 && k < n1) gFl[k] += q[4] * (1.0 - q[5]) * lib.lam2_d[k];
          if (k + 1 >= n0 && k + 1 < n1) gFl[k + 1] += q[4] * q[5] * lib.lam2_d[k + 1];
        } else {
          const double inv = 1.0 / q[1];
          for (int n = j0; n <= j1; ++n) {
            const double u = (lib.lnwave_d[n] - q[0]) * inv;
            gFl[n] += q[4] * exp(-0.5 * u * u) * lib.lam2_d[n];
          }
        }
      }
    }
  }
  __syncthreads();
  // ---------------- attenuation adjoint on the owned pixels (eq. D2)
  T *GY = (T *)a.GY + (size_t)r * a.N_pad, *GO = (T *)a.GO + (size_t)r * a.N_pad;
  const double Eb = 0.85 - 1.9 * pr.delta;
  for (int n = n0; n < n1; ++n) {
    const double l = lib.lnlv_d[n];
    const double p = exp(pr.alpha_bc * l), qd = exp(pr.delta * l);
    const double sh = lib.dust_a_d[n] + Eb * lib.dust_d_d[n];
    const double Tbc = exp(-pr.tau_bc * p), Td = exp(-pr.tau_diff * qd * sh);
    const double g = gFl[n];
    GY[n] = (T)(g * Td * Tbc);
    GO[n] = (T)(g * Td);
    const double ya = (double)Yr[n], fa = (double)Fr[n];
    gtb += g * ya * (-p);
    gab += g * ya * (-pr.tau_bc * p * l);
    gtd += g * fa * (-qd * sh);
    gdl += g * fa * (-pr.tau_diff * (qd * l * sh - 1.9 * qd * lib.dust_d_d[n]));
  }
  for (int n = N + tid; n < a.N_pad; n += 256) {
    GY[n] = (T)0;
    GO[n] = (T)0;
  }
  const double s_z = block_sum256(gz, red), s_lm = block_sum256(glm, red);
  const double s_tb = block_sum256(gtb, red), s_ab = block_sum256(gab, red);
  const double s_td = block_sum256(gtd, red), s_dl = block_sum256(gdl, red);
  if (tid == 0) {
    double *gb = a.gbuf + (size_t)r * 16;
    gb[GB_Z] = s_z;
    gb[GB_LOGMASS] = s_lm * 2.302585092994046;
    gb[GB_TAU_BC] = s_tb;
    gb[GB_ALPHA_BC] = s_ab;
    gb[GB_TAU_DIFF] = s_td;
    gb[GB_DELTA] = s_dl;
  }
}

// ---------------------------------------------------------------------------------
// dW[r][k] = sum_n G_seg(k)[r][n] L[k][n]; G_Y for young-segment columns, G_O for old.
// FP32: MFMA 32x32x2 with the reduction (wavelength) axis contiguous in both operands.
// ---------------------------------------------------------------------------------
template <int MT, int NT>
__global__ void __launch_bounds__(256) k_bwd_f32(const float *__restrict__ GY, const float *__restrict__ GO,
                                                 const float *__restrict__ Ln, int N_pad, int K_pad, int K_young_pad,
                                                 double *__restrict__ dW) {
  constexpr int KT = 32, LDSK = KT + 4, WM = 2, WN = 2;
  constexpr int WTM = MT / WM, WTN = NT / WN, BM = WTM / 32, BN = WTN / 32;
  constexpr int A4 = MT * KT / 4 / 256, B4 = NT * KT / 4 / 256;
  __shared__ __attribute__((aligned(16))) float As[MT * LDSK];
  __shared__ __attribute__((aligned(16))) float Bs[NT * LDSK];
  const int n_ct = K_pad / NT;
  const int mt = blockIdx.x / n_ct, ct = blockIdx.x % n_ct;
  const int m0 = mt * MT, c0 = ct * NT;
  const float *G = c0 < K_young_pad ? GY : GO;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN, li = lane & 31, lh = lane >> 5;
  // each 32-wide reduction tile is accumulated in FP32 and the tile partials are summed
  // in FP64, which keeps the differences dW[j+1] - dW[j] of the metallicity adjoint accurate
  double dacc[BM][BN][16];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) dacc[i][j][e] = 0.0;
  f32x4 ra[A4], rb[B4];
  const int nt = N_pad / KT;
#pragma unroll
  for (int q = 0; q < A4; ++q) {
    const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;
    ra[q] = *(const f32x4 *)(G + (size_t)(m0 + row) * N_pad + c4 * 4);
  }
#pragma unroll
  for (int q = 0; q < B4; ++q) {
    const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;
    rb[q] = *(const f32x4 *)(Ln + (size_t)(c0 + row) * N_pad + c4 * 4);
  }
  for (int t = 0; t < nt; ++t) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < A4; ++q) {
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;
      *(f32x4 *)(As + row * LDSK + c4 * 4) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < B4; ++q) {
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;
      *(f32x4 *)(Bs + row * LDSK + c4 * 4) = rb[q];
    }
    __syncthreads();
    if (t + 1 < nt) {
      const int k0 = (t + 1) * KT;
#pragma unroll
      for (int q = 0; q < A4; ++q) {
        const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;
        ra[q] = *(const f32x4 *)(G + (size_t)(m0 + row) * N_pad + k0 + c4 * 4);
      }
#pragma unroll
      for (int q = 0; q < B4; ++q) {
        const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;
        rb[q] = *(const f32x4 *)(Ln + (size_t)(c0 + row) * N_pad + k0 + c4 * 4);
      }
    }
    float af[BM][16], bf[BN][16];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      const float *p = As + (wm * WTM + i * 32 + li) * LDSK + lh * 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 v = *(const f32x4 *)(p + 4 * q);
        af[i][4 * q] = v[0]; af[i][4 * q + 1] = v[1]; af[i][4 * q + 2] = v[2]; af[i][4 * q + 3] = v[3];
      }
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const float *p = Bs + (wn * WTN + j * 32 + li) * LDSK + lh * 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 v = *(const f32x4 *)(p + 4 * q);
        bf[j][4 * q] = v[0]; bf[j][4 * q + 1] = v[1]; bf[j][4 * q + 2] = v[2]; bf[j][4 * q + 3] = v[3];
      }
    }
    v16f acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) dacc[i][j][e] += (double)acc[i][j][e];
  }
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = wm * WTM + i * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
      for (int j = 0; j < BN; ++j) dW[(size_t)(m0 + rl) * K_pad + c0 + wn * WTN + j * 32 + li] = dacc[i][j][e];
    }
}

// FP64: LDS-tiled FMA, dW = G L^T with L^T = LT64 [N_pad][K_pad]
__global__ void __launch_bounds__(256) k_bwd_f64(const double *__restrict__ GY, const double *__restrict__ GO,
                                                 const double *__restrict__ LT, int N_pad, int K_pad, int K_young_pad,
                                                 double *__restrict__ dW) {
  constexpr int MT = 64, NT = 64, KT = 16;
  __shared__ double As[MT][KT + 1];
  __shared__ double Bs[KT][NT + 1];
  const int n_ct = K_pad / NT;
  const int mt = blockIdx.x / n_ct, ct = blockIdx.x % n_ct;
  const int m0 = mt * MT, c0 = ct * NT;
  const double *G = c0 < K_young_pad ? GY : GO;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < N_pad; k0 += KT) {
    __syncthreads();
    for (int idx = tid; idx < MT * KT; idx += 256) {
      const int row = idx / KT, c = idx % KT;
      As[row][c] = G[(size_t)(m0 + row) * N_pad + k0 + c];
    }
    for (int idx = tid; idx < KT * NT; idx += 256) {
      const int row = idx / NT, c = idx % NT;
      Bs[row][c] = LT[(size_t)(k0 + row) * K_pad + c0 + c];
    }
    __syncthreads();
    for (int kk = 0; kk < KT; ++kk) {
      double av[4], bv[4];
      for (int i = 0; i < 4; ++i) av[i] = As[ty + 16 * i][kk];
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx + 16 * j];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) dW[(size_t)(m0 + ty + 16 * i) * K_pad + c0 + tx + 16 * j] = acc[i][j];
}

// ---------------------------------------------------------------------------------
// Weights / lines adjoint and the final gradient row.
// ---------------------------------------------------------------------------------
struct AdjPrepArgs {
  const double *theta;
  int P, B;
  const PointRow *rows;
  const void *dW;
  int f64;
  const int *kpos;
  int line_k0;
  const double *gbuf, *gnoise, *dLl;
  double *grad;
};

__global__ void __launch_bounds__(256) k_adj_prep(DevLib lib, AdjPrepArgs a) {
  extern __shared__ double sm[];
  const int K_pad = lib.K_pad, n = lib.n_sfh, na = lib.n_age, nz = lib.n_z, nf = lib.n_afe, ny = lib.n_young;
  double *gacc = sm;                    // [K_pad] d logL / d W
  double *wrow = gacc + K_pad;          // [K_pad] W (recomputed, lines only)
  double *edges = wrow + K_pad;         // [n+1]
  double *dT = edges + n + 1;           // [n+1]
  double *zt = dT + n + 1;              // [n]
  double *zd = zt + n;                  // [n] dt/dzeta
  double *gzeta = zd + n;               // [n]
  double *gm = gzeta + n;               // [n] d/d mass
  double *wq = gm + n;                  // [ny]
  double *gwq = wq + ny;                // [ny]
  double *red = gwq + ny;               // [256]
  int *zj = (int *)(red + 256);         // [n]
  __shared__ double s_sc[4];
  const int r = blockIdx.x, tid = threadIdx.x;
  const PointRow pr = a.rows[r];
  if (pr.b < 0) return;
  const double *th = a.theta + (size_t)pr.b * a.P;
  for (int k = tid; k < K_pad; k += 256) {
    gacc[k] = ((const double *)a.dW)[(size_t)r * K_pad + k];
    wrow[k] = 0.0;
  }
  const double z = pr.z, opz = 1.0 + z, t_univ = pr.t_univ;
  const double Ez = sqrt(lib.Om * opz * opz * opz + 1.0 - lib.Om);
  const double dt_dz = -(kMpc_km / lib.H0 / kYr_s) / (opz * Ez);
  const double lnR = log(t_univ / lib.T1);
  for (int i = tid; i <= n; i += 256) {
    double T, d = 0.0;
    if (i == 0) T = 0.0;
    else if (i == 1) T = lib.T1;
    else if (i == n) { T = t_univ; d = dt_dz; }
    else {
      const double e = (double)(i - 1) / (double)(n - 1);
      T = lib.T1 * exp(lnR * e);
      d = T * e * dt_dz / t_univ;
    }
    edges[i] = T;
    dT[i] = d;
  }
  const double *zh = th + TH_NSCALAR + n;
  for (int i = tid; i < n; i += 256) {
    double zeta;
    if (lib.n_zh == 0) zeta = th[TH_LOGZSOL];
    else if (i == 0) zeta = zh[0];
    else {
      const double x = ((double)i - 0.5) / (double)(n - 1) * (double)(lib.n_zh - 1);
      int k = (int)floor(x);
      if (k >= lib.n_zh - 1) k = lib.n_zh - 2;
      const double f = x - (double)k;
      zeta = zh[k] + f * (zh[k + 1] - zh[k]);
    }
    int j = 0;
    double t = 0.0;
    bool in = false;
    if (nz > 1) grid_split_dev(lib.logz, nz, zeta, j, t, in);
    zj[i] = j;
    zt[i] = t;
    zd[i] = (nz > 1 && in) ? 1.0 / (lib.logz[j + 1] - lib.logz[j]) : 0.0;
    gzeta[i] = 0.0;
    gm[i] = 0.0;
  }
  int ja = 0;
  double ta = 0.0, dta = 0.0;
  if (nf > 1) {
    bool in;
    grid_split_dev(lib.afe, nf, th[TH_AFE], ja, ta, in);
    dta = in ? 1.0 / (lib.afe[ja + 1] - lib.afe[ja]) : 0.0;
  }
  __syncthreads();
  const double *mass = th + TH_NSCALAR;

  // ---- lines: recompute the young weights and Q-weighted sums, then back to W and gas
  double ggz = 0.0, ggu = 0.0;
  if (lib.n_line > 0) {
    for (int ag = tid; ag < ny; ag += 256) {
      const double lo = lib.cell_lo[ag], hi = lib.cell_hi[ag];
      for (int i = 0; i < n && edges[i] < hi; ++i) {
        const double ov = fmin(hi, edges[i + 1]) - fmax(lo, edges[i]);
        if (ov <= 0.0) continue;
        const double w = mass[i] * ov / (edges[i + 1] - edges[i]);
        for (int q = 0; q < (nf > 1 ? 2 : 1); ++q) {
          const int ia = nf > 1 ? ja + q : 0;
          const double fa = nf > 1 ? (q == 0 ? 1.0 - ta : ta) : 1.0;
          if (nz > 1) {
            wrow[kpos_of(lib, ia, zj[i], ag)] += fa * (1.0 - zt[i]) * w;
            wrow[kpos_of(lib, ia, zj[i] + 1, ag)] += fa * zt[i] * w;
          } else {
            wrow[kpos_of(lib, ia, 0, ag)] += fa * w;
          }
        }
      }
      double s = 0.0;
      for (int ia = 0; ia < nf; ++ia)
        for (int m = 0; m < nz; ++m) s += wrow[kpos_of(lib, ia, m, ag)] * lib.Q[(ia * nz + m) * ny + ag];
      wq[ag] = s;
      gwq[ag] = 0.0;
    }
    __syncthreads();
    int jg = 0, ju = 0;
    double tg = 0.0, tu = 0.0;
    bool ig, iu;
    grid_split_dev(lib.zg, lib.n_zg, th[TH_GAS_LOGZ], jg, tg, ig);
    grid_split_dev(lib.un, lib.n_u, th[TH_GAS_LOGU], ju, tu, iu);
    const double dtg = ig ? 1.0 / (lib.zg[jg + 1] - lib.zg[jg]) : 0.0;
    const double dtu = iu ? 1.0 / (lib.un[ju + 1] - lib.un[ju]) : 0.0;
    const int nu = lib.n_u;
    // thread per age: sum over lines in a fixed order
    for (int ag = tid; ag < ny; ag += 256) {
      double gs = 0.0, gzg = 0.0, gu = 0.0;
      for (int l = 0; l < lib.n_line; ++l) {
        const double gL = pr.kind == 0 ? gacc[a.line_k0 + l] / kLsun : a.dLl[(size_t)r * lib.n_line + l];
        const size_t slab = (size_t)lib.n_line * ny;
        const double *tb = lib.line_table + (size_t)l * ny + ag;
        const double t00 = tb[(jg * nu + ju) * slab], t01 = tb[(jg * nu + ju + 1) * slab];
        const double t10 = tb[((jg + 1) * nu + ju) * slab], t11 = tb[((jg + 1) * nu + ju + 1) * slab];
        const double lh = (1 - tg) * (1 - tu) * t00 + (1 - tg) * tu * t01 + tg * (1 - tu) * t10 + tg * tu * t11;
        const double E = exp10(lh);
        gs += gL * E;
        const double gE = gL * wq[ag] * E * 2.302585092994046;
        gzg += gE * ((1 - tu) * (t10 - t00) + tu * (t11 - t01)) * dtg;
        gu += gE * ((1 - tg) * (t01 - t00) + tg * (t11 - t10)) * dtu;
      }
      gwq[ag] = gs;
      ggz += gzg;
      ggu += gu;
    }
    __syncthreads();
    for (int ag = tid; ag < ny; ag += 256)
      for (int ia = 0; ia < nf; ++ia)
        for (int m = 0; m < nz; ++m) gacc[kpos_of(lib, ia, m, ag)] += gwq[ag] * lib.Q[(ia * nz + m) * ny + ag];
    __syncthreads();
  }

  // ---- weights adjoint: thread per SFH bin, ages in increasing order
  double gz_e = 0.0, gafe = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double Ti = edges[i], Tj = edges[i + 1], dTb = Tj - Ti;
    int ag;
    {
      int l = 0, h = na;   // first cell whose upper edge exceeds Ti
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (lib.cell_hi[mid] > Ti) h = mid; else l = mid + 1;
      }
      ag = l;
    }
    double gmi = 0.0, gzi = 0.0;
    for (; ag < na && lib.cell_lo[ag] < Tj; ++ag) {
      const double lo = lib.cell_lo[ag], hi = lib.cell_hi[ag];
      const double upper = fmin(hi, Tj), lower = fmax(lo, Ti);
      const double ovr = upper - lower;
      if (ovr <= 0.0) continue;
      const double w = mass[i] * ovr / dTb;
      double gw = 0.0;
      for (int q = 0; q < (nf > 1 ? 2 : 1); ++q) {
        const int ia = nf > 1 ? ja + q : 0;
        const double fa = nf > 1 ? (q == 0 ? 1.0 - ta : ta) : 1.0;
        const double dfa = nf > 1 ? (q == 0 ? -dta : dta) : 0.0;
        double gA;
        if (nz > 1) {
          const double g0 = gacc[kpos_of(lib, ia, zj[i], ag)];
          const double g1 = gacc[kpos_of(lib, ia, zj[i] + 1, ag)];
          gA = (1.0 - zt[i]) * g0 + zt[i] * g1;
          gzi += fa * zd[i] * w * (g1 - g0);
        } else {
          gA = gacc[kpos_of(lib, ia, 0, ag)];
        }
        gw += fa * gA;
        gafe += dfa * w * gA;
      }
      gmi += gw * ovr / dTb;
      const double dov_i = (Ti > lo) ? -1.0 : 0.0;
      const double dov_j = (Tj < hi) ? 1.0 : 0.0;
      const double dw_i = mass[i] * (dov_i / dTb + ovr / (dTb * dTb));
      const double dw_j = mass[i] * (dov_j / dTb - ovr / (dTb * dTb));
      gz_e += gw * (dw_i * dT[i] + dw_j * dT[i + 1]);
    }
    gm[i] = gmi;
    gzeta[i] = gzi;
  }
  const double s_ze = block_sum256(gz_e, red);
  const double s_afe = block_sum256(gafe, red);
  const double s_gz = block_sum256(ggz, red);
  const double s_gu = block_sum256(ggu, red);
  double *gr = a.grad + (size_t)pr.b * a.P;
  for (int c = tid; c < a.P; c += 256) gr[c] = 0.0;
  __syncthreads();
  const double *gb = a.gbuf + (size_t)r * 16;
  for (int i = tid; i < n; i += 256) gr[TH_NSCALAR + i] = gm[i];
  if (tid == 0) {
    gr[TH_LOGMASS] = gb[GB_LOGMASS];
    gr[TH_ZRED] = gb[GB_Z] + s_ze;
    gr[TH_TAU_BC] = gb[GB_TAU_BC];
    gr[TH_ALPHA_BC] = gb[GB_ALPHA_BC];
    gr[TH_TAU_DIFF] = gb[GB_TAU_DIFF];
    gr[TH_DELTA] = gb[GB_DELTA];
    if (lib.n_line > 0) {
      gr[TH_GAS_LOGZ] = s_gz;
      gr[TH_GAS_LOGU] = s_gu;
    }
    if (nf > 1) gr[TH_AFE] = s_afe;
    for (int q = 0; q < 4; ++q) gr[TH_LOG_ERR_SCALE + q] = a.gnoise[(size_t)pr.b * 4 + q];
    // metallicity parameters: transpose of the bin interpolation (fixed order)
    if (lib.n_zh == 0) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += gzeta[i];
      gr[TH_LOGZSOL] = s;
    } else {
      double *gz = gr + TH_NSCALAR + n;
      gz[0] += gzeta[0];
      for (int i = 1; i < n; ++i) {
        const double x = ((double)i - 0.5) / (double)(n - 1) * (double)(lib.n_zh - 1);
        int k = (int)floor(x);
        if (k >= lib.n_zh - 1) k = lib.n_zh - 2;
        const double f = x - (double)k;
        gz[k] += (1.0 - f) * gzeta[i];
        gz[k + 1] += f * gzeta[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
sps_status run_adjoint(const sps_library *L, sps_obs *o, const double *theta, int B, int prec, double *grad,
                       hipStream_t s) {
  const DevLib &g = L->dev;
  Workspace &w = o->ws;
  const int B_pad = (B + kMAlign - 1) / kMAlign * kMAlign;
  const bool f64 = prec == SPS_FP64;
  if (g.N > 12288) return fail(SPS_E_SHAPE, "gradient pass supports up to 12288 wavelengths");
  AdjArgs aa;
  aa.theta = theta;
  aa.P = g.P;
  aa.B = B;
  aa.N_pad = g.N_pad;
  aa.n_line = g.n_line;
  aa.rows = w.rows;
  aa.obs_table = o->dev_obs;
  aa.F = w.F;
  aa.Yatt = w.Yatt;
  aa.gvec = w.gvec;
  aa.model = w.mbuf;
  aa.ld_g = o->host.n_data;
  aa.Lline = w.Lline;
  aa.scr = w.scr;
  aa.ld_scr = w.ld_scr;
  aa.GY = w.G;
  aa.GO = (char *)w.G + (size_t)B_pad * g.N_pad * (f64 ? 8 : 4);
  aa.gbuf = w.gbuf;
  aa.dLl = w.dLl;
  const size_t sm1 = (size_t)g.N * 8;
  static size_t attr1[2] = {0, 0};
  if (sm1 > 48 * 1024 && sm1 > attr1[f64 ? 1 : 0]) {
    const void *fn = f64 ? (const void *)k_adj_proj<double> : (const void *)k_adj_proj<float>;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm1) != hipSuccess)
      return fail(SPS_E_HIP, "hipFuncSetAttribute failed");
    attr1[f64 ? 1 : 0] = sm1;
  }
  (void)hipGetLastError();   // drop a stale code from an unrelated earlier HIP call of this thread
  if (f64) hipLaunchKernelGGL(k_adj_proj<double>, dim3(B), dim3(256), sm1, s, g, aa);
  else hipLaunchKernelGGL(k_adj_proj<float>, dim3(B), dim3(256), sm1, s, g, aa);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    if (f64) {
      hipLaunchKernelGGL(k_bwd_f64, dim3((B_pad / 64) * (g.K_pad / 64)), dim3(256), 0, s, (const double *)aa.GY,
                         (const double *)aa.GO, g.LT64, g.N_pad, g.K_pad, g.K_young_pad, (double *)w.dW);
    } else {
      hipLaunchKernelGGL((k_bwd_f32<128, 64>), dim3((B_pad / 128) * (g.K_pad / 64)), dim3(256), 0, s,
                         (const float *)aa.GY, (const float *)aa.GO, g.L32n, g.N_pad, g.K_pad, g.K_young_pad,
                         (double *)w.dW);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    AdjPrepArgs ap;
    ap.theta = theta;
    ap.P = g.P;
    ap.B = B;
    ap.rows = w.rows;
    ap.dW = w.dW;
    ap.f64 = f64 ? 1 : 0;
    ap.kpos = L->kpos_d;
    ap.line_k0 = L->line_k0;
    ap.gbuf = w.gbuf;
    ap.gnoise = w.gnoise;
    ap.dLl = w.dLl;
    ap.grad = grad;
    const size_t sm2 = sizeof(double) * (2 * (size_t)g.K_pad + 6 * (size_t)g.n_sfh + 2 + 2 * g.n_young + 256) +
                       sizeof(int) * (size_t)g.n_sfh + 64;
    if (sm2 > 150 * 1024) return fail(SPS_E_SHAPE, "gradient pass: library too large for one workgroup");
    static size_t attr2 = 0;
    if (sm2 > 48 * 1024 && sm2 > attr2) {
      if (hipFuncSetAttribute((const void *)k_adj_prep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm2) !=
          hipSuccess)
        return fail(SPS_E_HIP, "hipFuncSetAttribute failed");
      attr2 = sm2;
    }
    hipLaunchKernelGGL(k_adj_prep, dim3(B), dim3(256), sm2, s, g, ap);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(SPS_E_HIP, "gradient kernels failed: %s", hipGetErrorString(e));
  return SPS_OK;
}

}  // namespace sps
