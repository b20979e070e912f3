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
#include <type_traits>

#include "kernels.h"
#include "runtime.h"

namespace sps {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// nodes of the rows' span owned by one thread in the FP32 spectral transpose (the span is
// at most 256 * kAdjOwn nodes)
constexpr int kAdjOwn = 16;

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
  int fast;                     // FP32 path: per-node / per-pixel tables fit in LDS after gF
  int g_bytes;                  // bytes of the first dynamic LDS region (gF, or the span of rows)
  int nl_lds;                   // line slots of the line tables in LDS (spectra)
  int seg_cap;                  // FP32 spectra: bound on the rows' span in nodes
  double fr_max;                // photometry: largest |filter-node weight|
  int f_spans;                  // F and Yatt were formed only over the rows' spans (PointRow seg0 / seg_n)
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
  // dynamic LDS: [d logL / d F on the rest grid, N doubles (FP32 spectra: the span of the
  // rows in FP32, first f = F lambda^2, then d logL / d F)] [line tables, 5 x nl_lds
  // doubles] [FP32 path: per-node or per-pixel tables of the transpose]
  extern __shared__ __attribute__((aligned(16))) unsigned char adj_dyn[];
  double *gFl = (double *)adj_dyn;
  double *s_lnl = (double *)(adj_dyn + a.g_bytes), *s_sl = s_lnl + a.nl_lds, *s_dsl = s_sl + a.nl_lds;
  double *s_F = s_dsl + a.nl_lds, *s_T = s_F + a.nl_lds;
  unsigned char *xsm = (unsigned char *)(s_T + a.nl_lds);
  __shared__ double red[256];
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
  const bool fast_spec = sizeof(T) == 4 && a.fast && ob.kind != 0;
  if (!fast_spec)
    for (int n = n0; n < n1; ++n) gFl[n] = 0.0;
  int fs_seg0 = 0, fs_segn = 0;   // FP32 spectra: span of the rows, d logL / d F held there
  bool fx = false;                // FP32 photometry: d logL / d F held as fixed point,
  double fx_inv = 0.0, fx_scale = 0.0;   //   with this quantum (and its inverse, the scale)
  double gz = 0.0, glm = 0.0, gtb = 0.0, gab = 0.0, gtd = 0.0, gdl = 0.0;
  for (int i = tid; i < ob.n_data; i += 256) glm += gm[i] * mm[i];

  if (ob.kind == 0 && sizeof(T) == 4 && a.fast) {
    // ---------------- photometry, FP32 path: one thread per filter node over all bands
    // (the band from the offsets held in LDS), the node's interval found as in the
    // forward pass; per-node interval and weights kept in LDS for the transpose
    const double A = kC_cms * pr.scale_fnu / (opz * opz * kAng_cm * kAng_cm);
    const double dlnA = -1.0 / opz - 2.0 * ddl / pr.dl;
    const double lnopz = log1p(z);
    const double wlo = lib.wave_d[0], whi = lib.wave_d[N - 1];
    const int nfn = ob.n_fnodes, nb = ob.n_band;
    int *s_bo = (int *)xsm;
    for (int b = tid; b <= nb; b += 256) s_bo[b] = ob.band_off[b];
    double gmax = 0.0;
    for (int b = tid; b < nb; b += 256) {
      gz += gm[b] * dlnA * mm[b];
      gmax = fmax(gmax, fabs(gm[b]));
    }
    for (int o = 32; o > 0; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
    if ((tid & 63) == 0) red[tid >> 6] = gmax;
    __syncthreads();
    // every node adds its two shares (FP64 products) to d logL / d F as 64-bit fixed point
    // (LDS integer atomics), so the sums do not depend on the order of the additions.  The
    // scale bounds every share, |g_b| A |R_j|, below 2^(62 - hb), hb the bit length of nfn,
    // which leaves headroom for all shares landing on one pixel; the quantum is 2^-50 of
    // that bound at nfn = 2560.
    {
      const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * fabs(A) * a.fr_max;
      const int e = m > 0.0 ? max(ilogb(m) + 1, -960) : 0;   // scale and quantum stay normal
      const int hb = 32 - __clz(nfn);
      fx_scale = ldexp(1.0, 62 - hb - e);
      fx_inv = ldexp(1.0, e + hb - 62);
      fx = true;
    }
    unsigned long long *gi = (unsigned long long *)gFl;
    // ten nodes per thread per round: their node data, then their grid intervals and model
    // values, each group of loads in flight together (clamped indices); gz in node order
    constexpr int UJ = 10;
    for (int jb = tid; jb < nfn; jb += 256 * UJ) {
      double fwq[UJ], frq[UJ], lnq[UJ];
      int bq[UJ];
#pragma unroll
      for (int u = 0; u < UJ; ++u) {
        const int j = min(jb + 256 * u, nfn - 1);
        fwq[u] = ob.fw[j];
        frq[u] = ob.fr_d[j];
        lnq[u] = ob.fwln[j];
        int lo = 0, hi = nb - 1;   // band of node j: the last b with band_off[b] <= j
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_bo[mid] <= j) lo = mid; else hi = mid - 1;
        }
        bq[u] = lo;
      }
      double gq[UJ], w0q[UJ], w1q[UJ];
      float f0q[UJ], f1q[UJ];
      int kq[UJ];
#pragma unroll
      for (int u = 0; u < UJ; ++u) {
        // as the forward pass of the gradient pass (linear in lambda, the interval from the
        // node's log index on a log-uniform grid)
        const int k = min(max((int)floor((lnq[u] - lnopz - lib.lnw0) * lib.inv_dlnw), 0), N - 2);
        kq[u] = k;
        gq[u] = gm[bq[u]];
        w0q[u] = lib.wave_d[k];
        w1q[u] = lib.wave_d[k + 1];
        f0q[u] = (float)Fr[k];
        f1q[u] = (float)Fr[k + 1];
      }
#pragma unroll
      for (int u = 0; u < UJ; ++u) {
        const int j = jb + 256 * u;
        const double lr = fwq[u] / opz;
        const double coef = gq[u] * A * frq[u];
        if (j < nfn && lr >= wlo && lr <= whi) {   // nodes outside the model grid add nothing
          const double w0 = w0q[u], dw = w1q[u] - w0;
          const double t = (lr - w0) / dw;
          gz += coef * (((double)f1q[u] - (double)f0q[u]) / dw) * (-fwq[u] / (opz * opz));
          const int k = kq[u];
          const long long q0 = llrint(coef * (1.0 - t) * fx_scale), q1 = llrint(coef * t * fx_scale);
          if (q0 != 0) atomicAdd(gi + k, (unsigned long long)q0);
          if (q1 != 0) atomicAdd(gi + k + 1, (unsigned long long)q1);
        }
      }
    }
  } else if (ob.kind == 0) {
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
  } else if (fast_spec) {
    // ---------------- spectrum, FP32 path on a log-uniform rest grid: f = F lambda^2 over
    // the span of the rows staged in LDS; per pixel, the row's Gaussian weights by the
    // recurrence of the forward pass (w_{j+1} = w_j q_j, q_{j+1} = q_j e^{-h^2}); the
    // transpose gathers, for each owned node, the rows that cover it in pixel order
    const double S = pr.scale_fnu;
    const double dlnS = 1.0 / opz - 2.0 * ddl / pr.dl;
    const double lnopz = log1p(z);
    const int np = ob.n_data;
    const double lnw0 = lib.lnwave_d[0], lnw1 = lib.lnwave_d[N - 1];
    const double dln = 1.0 / lib.inv_dlnw;
    short *s_j0 = (short *)xsm, *s_j1 = s_j0 + np;
    float *s_cf = (float *)(xsm + ((4 * (size_t)np + 15) & ~(size_t)15));
    float *s_a0 = s_cf + np, *s_h = s_a0 + np;
    int *s_first = (int *)(s_h + np), *s_last = s_first + 256;
    // ln lambda of every 16th pixel, on the next 8-byte boundary (the host sizing leaves the slack)
    double *s_lp16 = (double *)(((uintptr_t)(s_last + 256) + 7) & ~(uintptr_t)7);
    // the row's span as the weight builder set it (common.h: spec_span); at least one node,
    // so that a row with a non-finite redshift still has owners in the transpose
    const int seg0 = pr.seg0;
    const int seg_n = max(min(pr.seg_n, a.seg_cap), 1);
    fs_seg0 = seg0;
    fs_segn = seg_n;
    float *seg = (float *)gFl;
    for (int k0 = tid; k0 < seg_n; k0 += 256 * 8) {   // eight loads per thread in flight
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + 256 * q;
        v[q] = k < seg_n ? (float)Fr[seg0 + k] * (float)lib.lam2_d[seg0 + k] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + 256 * q < seg_n) seg[k0 + 256 * q] = v[q];
    }
    s_first[tid] = INT_MAX;
    s_last[tid] = -1;
    __syncthreads();
    const int chunk_s = (seg_n + 255) / 256;   // nodes per owner in the transpose
    // the next pixel's inputs are requested while the current row is summed
    double gm_n = gm[min(tid, np - 1)], lp_n = ob.lnpix[min(tid, np - 1)], ks_n = ob.ksig[min(tid, np - 1)];
    for (int i = tid; i < np; i += 256) {
      const double gc = gm_n / kFnuAB;
      const double lpi = lp_n, ksi = ks_n;
      {
        const int inx = min(i + 256, np - 1);
        gm_n = gm[inx];
        lp_n = ob.lnpix[inx];
        ks_n = ob.ksig[inx];
      }
      if ((i & 15) == 0) s_lp16[i >> 4] = lpi;
      const double x = lpi - lnopz;
      int j0 = 1, j1 = 0;   // empty row
      float cf = 0.f, a0 = 0.f, hh = 0.f;
      if (x >= lnw0 && x <= lnw1) {
        // the forward pass's row on the log-uniform grid: position ux in node units,
        // width rs; nodes j0..j1 within five widths, or two nodes when the row is
        // narrower than half a node spacing
        const double s = ksi;
        const double ux = (x - lnw0) * lib.inv_dlnw;
        if (s < 0.5 * dln) {   // linear row on nodes k, k+1 (marked by h = 0, t kept in a0)
          const int k = min((int)floor(ux), N - 2);
          const float t = (float)(ux - (double)k);
          const double fk = seg[k - seg0], fk1 = seg[k + 1 - seg0];
          const double cont = fk + (double)t * (fk1 - fk);
          gz += gc * (dlnS * S * cont + S * (fk1 - fk) * (-lib.inv_dlnw / opz));
          j0 = k;
          j1 = k + 1;
          cf = (float)(gc * S);
          a0 = t;
        } else {
          const double rs = s * lib.inv_dlnw;
          j0 = max((int)ceil(ux - 5.0 * rs), 0);
          j1 = min((int)floor(ux + 5.0 * rs), N - 1);
          const float hf = 1.f / (float)rs, u0 = (float)((double)j0 - ux) * hf;
          float w = expf(-0.5f * u0 * u0), q = expf(-u0 * hf - 0.5f * hf * hf);
          const float c = expf(-hf * hf);
          float G = 0.f, num = 0.f, sug = 0.f, sugf = 0.f;
          const float *gp = seg + (j0 - seg0);
          const int nt = j1 - j0 + 1;
          int jj = 0;
          for (; jj + 8 <= nt; jj += 8) {   // eight taps per step: LDS reads ahead of the recurrence
            float g8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) g8[e] = gp[jj + e];
            if (jj > 0) {   // restarted from the exact Gaussian every step, as in the forward pass
              const float a = u0 + (float)jj * hf;
              w = expf(-0.5f * a * a);
              q = expf(-a * hf - 0.5f * hf * hf);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float uw = fmaf((float)(jj + e), hf, u0) * w;
              G += w;
              num += w * g8[e];
              sug += uw;
              sugf += uw * g8[e];
              w *= q;
              q *= c;
            }
          }
          for (; jj < nt; ++jj) {
            const float fj = gp[jj];
            const float uw = fmaf((float)jj, hf, u0) * w;
            G += w;
            num += w * fj;
            sug += uw;
            sugf += uw * fj;
            w *= q;
            q *= c;
          }
          // d g / d z = -u g / (s (1+z)) summed over the row, with and without f
          const double inv = 1.0 / s;
          const double Gd = G, cont = (double)num / Gd;
          const double dg = (double)sug * (-inv / opz), dgf = (double)sugf * (-inv / opz);
          gz += gc * (dlnS * S * cont + S * (dgf - cont * dg) / Gd);
          cf = (float)(gc * S / Gd);
          a0 = u0;
          hh = hf;
        }
        const int c_lo = max(j0 - seg0, 0) / chunk_s, c_hi = min(j1 - seg0, seg_n - 1) / chunk_s;
        for (int cc = c_lo; cc <= c_hi; ++cc) {   // owners whose nodes this row covers
          atomicMin(&s_first[cc], i);
          atomicMax(&s_last[cc], i);
        }
      }
      s_j0[i] = (short)j0;
      s_j1[i] = (short)j1;
      s_cf[i] = cf;
      s_a0[i] = a0;
      s_h[i] = hh;
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
      // pixels within 10 sigma of a line, split over two threads per line when the lines
      // fit, halves added in a fixed order
      const int tpl = nl <= 128 ? 2 : 1;
      for (int l0 = tid; l0 < nl * tpl; l0 += 256) {
        const int l = l0 / tpl, part = l0 - l * tpl;
        const double mu = s_lnl[l], sl = s_sl[l];
        const double vhi = mu + 10.0 * sl;
        // the pixels within 10 sigma: [ia, ib) with ia the first ln lambda >= mu - 10 sl and
        // ib the first > mu + 10 sl, each by bisection on every 16th pixel in LDS, then the
        // (at most 15) candidates of that block, loaded together
        const int nc = (np + 15) >> 4;
        auto first_pix = [&](double v, bool strict) {   // first i with lnpix[i] >= v (> v if strict)
          int lo = 0, hi = nc;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (strict ? s_lp16[mid] <= v : s_lp16[mid] < v) lo = mid + 1; else hi = mid;
          }
          const int b0 = max(16 * (lo - 1) + 1, 0), b1 = min(16 * lo, np);
          int cnt = 0;
#pragma unroll
          for (int e = 0; e < 15; ++e) {
            const double x = ob.lnpix[min(b0 + e, np - 1)];
            cnt += (b0 + e < b1) && (strict ? x <= v : x < v);
          }
          return b0 + cnt;
        };
        const int ia = first_pix(mu - 10.0 * sl, false);
        const int ib = max(first_pix(vhi, true), ia);
        const int im = ia + (ib - ia + 1) / 2;
        const int i0 = tpl == 1 ? ia : (part == 0 ? ia : im), i1 = tpl == 1 ? ib : (part == 0 ? im : ib);
        double gFlx = 0.0, gzl = 0.0;
        const double isl = 1.0 / sl, nrm = isl / 2.5066282746310002, gscale = kAng_cm / (kFnuAB * kC_cms);
        const double zf = s_F[l] * isl / opz, df = s_F[l] * isl * s_dsl[l];
        constexpr int LB = 16;   // pixels whose loads are in flight together (clamped)
        for (int ib8 = i0; ib8 < i1; ib8 += LB) {
          double lpq[LB], gq[LB], pq[LB];
#pragma unroll
          for (int e = 0; e < LB; ++e) {
            const int i = min(ib8 + e, np - 1);
            lpq[e] = ob.lnpix[i];
            gq[e] = gm[i];
            pq[e] = ob.pix[i];
          }
#pragma unroll
          for (int e = 0; e < LB; ++e) {
            if (ib8 + e >= i1) break;
            const double u = (lpq[e] - mu) * isl;
            const double Nn = (double)expf((float)(-0.5 * u * u)) * nrm;
            const double glp = gq[e] * pq[e] * gscale;
            gFlx += glp * Nn;
            gzl += glp * Nn * (u * zf + (u * u - 1.0) * df);
          }
        }
        if (tpl == 2) {
          const double of = __shfl_xor(gFlx, 1, 64), oz = __shfl_xor(gzl, 1, 64);
          gFlx = part == 0 ? gFlx + of : of + gFlx;
          gzl = part == 0 ? gzl + oz : oz + gzl;
          if (part != 0) continue;
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
    __syncthreads();   // the rows no longer read f: the span now receives d logL / d F
    {
      // each thread owns at most kAdjOwn consecutive nodes of the span and adds, in pixel
      // order, the rows that cover them into one register per owned node (as many
      // registers as the owner size rounded up to 8, 12 or 16), then writes its nodes
      // once.  A row's weight at node j is the Gaussian 2^(u^2 log2(e) / -2), u = (j - j0) h
      // + a0, one hardware exp2 per node (the row normalisation G is the forward's).
      const int c0 = tid * chunk_s, c1 = min(c0 + chunk_s, seg_n);
      auto owner = [&](auto own_c) {
        constexpr int OWN = decltype(own_c)::value;
        const int na0 = seg0 + c0, na1 = seg0 + c1 - 1;   // owned nodes
        float acc[OWN];
#pragma unroll
        for (int e = 0; e < OWN; ++e) acc[e] = 0.f;
        for (int i = s_first[tid]; i <= s_last[tid]; ++i) {
          const int j0 = s_j0[i], j1 = s_j1[i];
          if (max(j0, na0) > min(j1, na1)) continue;
          const float cf = s_cf[i], hf = s_h[i], a0 = s_a0[i];
          const int lo = j0 - na0, hi = j1 - na0;   // the row's nodes as owned offsets
          if (hf == 0.f) {   // linear row on nodes j0 = k, j1 = k + 1 (a0 holds t)
#pragma unroll
            for (int e = 0; e < OWN; ++e) acc[e] += (e == lo ? cf * (1.f - a0) : 0.f) + (e == hi ? cf * a0 : 0.f);
          } else {
            const float ub = fmaf((float)(na0 - j0), hf, a0);   // u at the first owned node
#pragma unroll
            for (int e = 0; e < OWN; ++e) {
              const float u = fmaf((float)e, hf, ub);
              const float w = __builtin_amdgcn_exp2f(u * u * -0.72134752044448170f);
              acc[e] += e >= lo && e <= hi ? cf * w : 0.f;
            }
          }
        }
#pragma unroll
        for (int e = 0; e < OWN; ++e)
          if (c0 + e < c1) seg[c0 + e] = acc[e];
      };
      if (c0 < c1) {
        if (chunk_s <= 8) owner(std::integral_constant<int, 8>{});
        else if (chunk_s <= 12) owner(std::integral_constant<int, 12>{});
        else owner(std::integral_constant<int, kAdjOwn>{});
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
  // gF is complete after the barrier: a coalesced pass, eight nodes per thread with all
  // their loads in flight (clamped indices); each thread's sums still run in node order.
  // d logL / d F is zero outside the row's span; where the forward pass formed F and the
  // young part only over the rows' spans they are not read there (G = 0 is written)
  const int sp_lo = a.f_spans ? pr.seg0 : 0, sp_hi = a.f_spans ? pr.seg0 + pr.seg_n : N;
  for (int nb = tid; nb < N; nb += 256 * 8) {
    double lq[8], gq[8], ddq[8], yq[8], fq[8];
    float lfq[8], daq[8], dfq[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int n = min(max(nb + 256 * u, sp_lo), max(sp_hi - 1, 0));
      lq[u] = lib.lnlv_d[n];
      ddq[u] = lib.dust_d_d[n];
      yq[u] = (double)Yr[n];
      fq[u] = (double)Fr[n];
      if (fx) gq[u] = (double)(long long)((const unsigned long long *)gFl)[n] * fx_inv;
      else if (!fast_spec) gq[u] = gFl[n];
      else gq[u] = (n >= fs_seg0 && n < fs_seg0 + fs_segn) ? (double)((const float *)gFl)[n - fs_seg0] * lib.lam2_d[n]
                                                           : 0.0;
      if (sizeof(T) == 4) {
        lfq[u] = lib.lnlv_f[n];
        daq[u] = lib.dust_a_f[n];
        dfq[u] = lib.dust_d_f[n];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int n = nb + 256 * u;
      if (n >= N) break;
      if (n < sp_lo || n >= sp_hi) {
        GY[n] = (T)0;
        GO[n] = (T)0;
        continue;
      }
      const double l = lq[u], g = gq[u];
      double p, qd, sh, Tbc, Td;
      if (sizeof(T) == 4) {   // FP32 path: the factors in FP32, as the forward epilogue forms them
        const float lf = lfq[u];
        const float pf = expf((float)pr.alpha_bc * lf), qf = expf((float)pr.delta * lf);
        const float shf = daq[u] + (float)Eb * dfq[u];
        p = pf;
        qd = qf;
        sh = shf;
        Tbc = expf(-(float)pr.tau_bc * pf);
        Td = expf(-(float)pr.tau_diff * qf * shf);
      } else {
        p = exp(pr.alpha_bc * l);
        qd = exp(pr.delta * l);
        sh = lib.dust_a_d[n] + Eb * ddq[u];
        Tbc = exp(-pr.tau_bc * p);
        Td = exp(-pr.tau_diff * qd * sh);
      }
      GY[n] = (T)(g * Td * Tbc);
      GO[n] = (T)(g * Td);
      const double ya = yq[u], fa = fq[u];
      gtb += g * ya * (-p);
      gab += g * ya * (-pr.tau_bc * p * l);
      gtd += g * fa * (-qd * sh);
      gdl += g * fa * (-pr.tau_diff * (qd * l * sh - 1.9 * qd * ddq[u]));
    }
  }
  for (int n = N + tid; n < a.N_pad; n += 256) {
    GY[n] = (T)0;
    GO[n] = (T)0;
  }
  // six block sums at once: wave butterflies, then the four waves in a fixed order
  double v6[6] = {gz, glm, gtb, gab, gtd, gdl};
#pragma unroll
  for (int k = 0; k < 6; ++k)
    for (int o = 32; o > 0; o >>= 1) v6[k] += __shfl_xor(v6[k], o, 64);
  __syncthreads();
  if ((tid & 63) == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[(tid >> 6) * 6 + k] = v6[k];
  __syncthreads();
  const double s_z = (red[0] + red[6]) + (red[12] + red[18]), s_lm = (red[1] + red[7]) + (red[13] + red[19]);
  const double s_tb = (red[2] + red[8]) + (red[14] + red[20]), s_ab = (red[3] + red[9]) + (red[15] + red[21]);
  const double s_td = (red[4] + red[10]) + (red[16] + red[22]), s_dl = (red[5] + red[11]) + (red[17] + red[23]);
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
// With n_split = 2 the wavelength tiles are halved between two blocks per output tile,
// which write dW and dW + split_stride; the weight-builder adjoint adds the two halves.
// With rows given (a log-uniform grid), G is zero outside each row's rest-frame span
// (PointRow seg0 / seg_n: the span under the filters for photometry, the pixels' rest
// range widened by the LSF rows for spectra); the block's wavelength range is the union
// of its rows' spans (two nodes of margin each side), the whole grid if a row has none.
// ---------------------------------------------------------------------------------
template <int MT, int NT>
__global__ void __launch_bounds__(256) k_bwd_f32(const float *__restrict__ GY, const float *__restrict__ GO,
                                                 const float *__restrict__ Ln, int N_pad, int K_pad, int K_young_pad,
                                                 const uint32_t *__restrict__ rowmask, int mask_words,
                                                 double *__restrict__ dW, int n_split, size_t split_stride,
                                                 const PointRow *__restrict__ rows) {
  constexpr int KT = 32, LDSK = KT + 4, WM = 2, WN = 2;
  constexpr int WTM = MT / WM, WTN = NT / WN, BM = WTM / 32, BN = WTN / 32;
  constexpr int A4 = MT * KT / 4 / 256, B4 = NT * KT / 4 / 256;
  __shared__ __attribute__((aligned(16))) float As[2][MT * LDSK];
  __shared__ __attribute__((aligned(16))) float Bs[2][NT * LDSK];
  __shared__ uint32_t s_any;
  __shared__ int s_lo, s_hi, s_full;
  const int n_ct = K_pad / NT;
  const int tile = blockIdx.x / n_split, half = blockIdx.x - tile * n_split;
  const int mt = tile / n_ct, ct = tile % n_ct;
  dW += half * split_stride;
  const int m0 = mt * MT, c0 = ct * NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN, li = lane & 31, lh = lane >> 5;
  // a column tile whose weights are zero in every row of the block needs no product: the
  // rows' occupancy bits (32-wide K tiles) decide, and the block writes zeros
  if (tid == 0) {
    s_any = 0u;
    s_lo = INT_MAX;
    s_hi = 0;
    s_full = rows ? 0 : 1;
  }
  __syncthreads();
  if (rows && tid < MT) {
    const PointRow &pr = rows[m0 + tid];
    if (pr.b >= 0) {
      if (pr.seg_n > 0) {
        atomicMin(&s_lo, pr.seg0 - 2);
        atomicMax(&s_hi, pr.seg0 + pr.seg_n + 2);
      } else {
        s_full = 1;
      }
    }
  }
  if (rowmask) {
    uint32_t any = 0u;
    for (int rr = tid; rr < MT; rr += 256)
      for (int t32 = c0 / 32; t32 < (c0 + NT) / 32; ++t32)
        any |= (rowmask[(size_t)(m0 + rr) * mask_words + (t32 >> 5)] >> (t32 & 31)) & 1u;
    if (any) s_any = 1u;
  } else if (tid == 0) {
    s_any = 1u;
  }
  __syncthreads();
  if (s_any == 0u) {
    for (int idx = tid; idx < MT * NT; idx += 256) dW[(size_t)(m0 + idx / NT) * K_pad + c0 + idx % NT] = 0.0;
    return;
  }
  const float *G = c0 < K_young_pad ? GY : GO;
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
  const int nt_all = N_pad / KT;
  int t_lo = 0, t_hi = nt_all;   // wavelength tiles where some row's G can be nonzero
  if (!s_full) {
    t_lo = min(max(s_lo, 0) / KT, nt_all);
    t_hi = max(min((s_hi + KT - 1) / KT, nt_all), t_lo);
  }
  const int ta = t_lo + (t_hi - t_lo) * half / n_split, nt = t_lo + (t_hi - t_lo) * (half + 1) / n_split;
#define SPS_BWD_LOAD(k0_)                                                                  \
  {                                                                                        \
    _Pragma("unroll") for (int q = 0; q < A4; ++q) {                                       \
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;                         \
      ra[q] = *(const f32x4 *)(G + (size_t)(m0 + row) * N_pad + (k0_) + c4 * 4);           \
    }                                                                                      \
    _Pragma("unroll") for (int q = 0; q < B4; ++q) {                                       \
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;                         \
      rb[q] = *(const f32x4 *)(Ln + (size_t)(c0 + row) * N_pad + (k0_) + c4 * 4);          \
    }                                                                                      \
  }
#define SPS_BWD_STORE(buf_)                                                                \
  {                                                                                        \
    _Pragma("unroll") for (int q = 0; q < A4; ++q) {                                       \
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;                         \
      *(f32x4 *)(As[buf_] + row * LDSK + c4 * 4) = ra[q];                                  \
    }                                                                                      \
    _Pragma("unroll") for (int q = 0; q < B4; ++q) {                                       \
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;                         \
      *(f32x4 *)(Bs[buf_] + row * LDSK + c4 * 4) = rb[q];                                  \
    }                                                                                      \
  }
  if (ta < nt) {   // an empty range leaves this half's dW zero
    SPS_BWD_LOAD(ta * KT);
    SPS_BWD_STORE(0);
  }
  // double-buffered: the tile t + 1 is loaded into registers during the products of tile
  // t and stored into the other buffer, whose last readers finished before the barrier
  for (int t = ta; t < nt; ++t) {
    const int buf = (t - ta) & 1;
    SPS_BWD_LOAD(min(t + 1, nt - 1) * KT);
    __syncthreads();
    float af[BM][16], bf[BN][16];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      const float *p = As[buf] + (wm * WTM + i * 32 + li) * LDSK + lh * 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 v = *(const f32x4 *)(p + 4 * q);
        af[i][4 * q] = v[0]; af[i][4 * q + 1] = v[1]; af[i][4 * q + 2] = v[2]; af[i][4 * q + 3] = v[3];
      }
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const float *p = Bs[buf] + (wn * WTN + j * 32 + li) * LDSK + lh * 16;
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
    SPS_BWD_STORE(buf ^ 1);
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) dacc[i][j][e] += (double)acc[i][j][e];
  }
#undef SPS_BWD_LOAD
#undef SPS_BWD_STORE
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
  const double *dW2;   // second half of the FP32 dW split over wavelengths, or NULL
  int f64;
  const int *kpos;
  int line_k0;
  const double *gbuf, *gnoise, *dLl;
  double *grad;
};

// LDS layout of k_adj_prep, in doubles.  The young-weight row is dead once the
// photon-weighted sums are formed; its space then holds the reduction partials.
struct AdjPrepSmem {
  int gacc, wrow, red, tab, edges, dT, mass, mr, zt, zd, zf, gzeta, wq, gwq, zj, zk, total;
  __host__ __device__ AdjPrepSmem(const DevLib &lib) {
    const int n = lib.n_sfh, ny = lib.n_young;
    const int nw = lib.n_line > 0 ? ny * lib.n_z * lib.n_afe : 0;
    const int nr = 8 * ny > 16 ? 8 * ny : 16;
    int o = 0;
    gacc = o;  o += lib.K_pad;                   // d logL / d W
    wrow = o;  red = o;  o += nw > nr ? nw : nr; // young SSP weights; later the partials
    tab = o;   o += prep_tab_len(lib);           // node tables
    edges = o; o += n + 1;
    dT = o;    o += n + 1;                       // d T_i / d z
    mass = o;  o += n;
    mr = o;    o += n;                           // bin mass per unit time
    zt = o;    o += n;
    zd = o;    o += n;                           // d t / d zeta
    zf = o;    o += n;                           // bin -> history-node interpolation weight
    gzeta = o; o += n;
    wq = o;    o += ny;
    gwq = o;   o += ny;
    zj = o;    o += (n + 1) / 2;                 // int: metallicity bracket
    zk = o;    o += (n + 1) / 2;                 // int: history node
    total = o;
  }
};

// bracketing node j, fraction t and whether x lies inside the grid, on a short grid held
// in LDS (the clamped split of grid_split_dev, by bisection)
__device__ __forceinline__ void split_in_lds(const double *nodes, int n, double x, int &j, double &t, bool &inside) {
  inside = x >= nodes[0] && x <= nodes[n - 1];
  const double xc = fmin(fmax(x, nodes[0]), nodes[n - 1]);
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (nodes[mid] <= xc) lo = mid; else hi = mid;
  }
  j = lo;
  t = (xc - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
}

// One workgroup per sorted row.  The node tables and the row of d logL / d W are copied
// to LDS first (all loads in flight together); every search then runs in LDS.
__global__ void __launch_bounds__(256, 4) k_adj_prep(DevLib lib, AdjPrepArgs a) {
  extern __shared__ double sm[];
  const AdjPrepSmem S(lib);
  const int K_pad = lib.K_pad, n = lib.n_sfh, na = lib.n_age, nz = lib.n_z, nf = lib.n_afe, ny = lib.n_young;
  const int nl = lib.n_line;
  double *gacc = sm + S.gacc, *wrow = sm + S.wrow, *tab = sm + S.tab;
  const double *t_logz = tab, *t_afe = tab + nz, *s_clo = tab + nz + nf, *s_chi = s_clo + na;
  const double *s_zg = s_chi + na, *s_un = s_zg + lib.n_zg, *s_Q = s_un + lib.n_u;
  double *edges = sm + S.edges, *dT = sm + S.dT, *mass = sm + S.mass, *mr = sm + S.mr, *zt = sm + S.zt;
  double *zd = sm + S.zd, *zf = sm + S.zf, *gzeta = sm + S.gzeta, *wq = sm + S.wq, *gwq = sm + S.gwq;
  double *red = sm + S.red;
  int *zj = (int *)(sm + S.zj), *zk = (int *)(sm + S.zk);
  const int r = blockIdx.x, tid = threadIdx.x;
  const PointRow pr = a.rows[r];
  if (pr.b < 0) return;
  double *gr = a.grad + (size_t)pr.b * a.P;
  const double *th = a.theta + (size_t)pr.b * a.P;

  // ---- the row of d logL / d W, the node-table block and the bin masses to LDS
  {
    const double2 *g2 = (const double2 *)((const double *)a.dW + (size_t)r * K_pad);   // K_pad even
    // FP32 pass: dW in two wavelength halves, added here (first half + second half)
    const double2 *h2 = a.dW2 ? (const double2 *)(a.dW2 + (size_t)r * K_pad) : nullptr;
    const double2 *t2 = (const double2 *)lib.prep_tab;                                  // even length
    const int ng2 = K_pad >> 1, nt2 = prep_tab_len(lib) >> 1;
    double2 vg[5], vt[2];
    double vm;
#pragma unroll
    for (int u = 0; u < 5; ++u) vg[u] = g2[min(tid + 256 * u, ng2 - 1)];
    if (h2) {
      double2 vh[5];
#pragma unroll
      for (int u = 0; u < 5; ++u) vh[u] = h2[min(tid + 256 * u, ng2 - 1)];
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        vg[u].x += vh[u].x;
        vg[u].y += vh[u].y;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) vt[u] = t2[min(tid + 256 * u, nt2 - 1)];
    vm = th[TH_NSCALAR + min(tid, n - 1)];
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int i = tid + 256 * u;
      if (i < ng2) {
        gacc[2 * i] = vg[u].x;
        gacc[2 * i + 1] = vg[u].y;
      }
    }
    for (int i = tid + 256 * 5; i < ng2; i += 256) {
      double2 v = g2[i];
      if (h2) {
        const double2 vh = h2[i];
        v.x += vh.x;
        v.y += vh.y;
      }
      gacc[2 * i] = v.x;
      gacc[2 * i + 1] = v.y;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + 256 * u;
      if (i < nt2) {
        tab[2 * i] = vt[u].x;
        tab[2 * i + 1] = vt[u].y;
      }
    }
    for (int i = tid + 256 * 2; i < nt2; i += 256) {
      const double2 v = t2[i];
      tab[2 * i] = v.x;
      tab[2 * i + 1] = v.y;
    }
    if (tid < n) mass[tid] = vm;
    for (int i = tid + 256; i < n; i += 256) mass[i] = th[TH_NSCALAR + i];
    for (int c = tid; c < a.P; c += 256) gr[c] = 0.0;   // every column not written below is 0
    if (nl > 0)
      for (int k = tid; k < ny * nz * nf; k += 256) wrow[k] = 0.0;
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
  __syncthreads();

  // ---- bin metallicities and their brackets; alpha bracket
  const double *zh = th + TH_NSCALAR + n;
  for (int i = tid; i < n; i += 256) {
    double zeta;
    int k = 0;
    double f = 0.0;
    if (lib.n_zh == 0) zeta = th[TH_LOGZSOL];
    else if (i == 0) zeta = zh[0];
    else {
      const double x = ((double)i - 0.5) / (double)(n - 1) * (double)(lib.n_zh - 1);
      k = (int)floor(x);
      if (k >= lib.n_zh - 1) k = lib.n_zh - 2;
      f = x - (double)k;
      zeta = zh[k] + f * (zh[k + 1] - zh[k]);
    }
    int j = 0;
    double t = 0.0;
    bool in = false;
    if (nz > 1) split_in_lds(t_logz, nz, zeta, j, t, in);
    zj[i] = j;
    zt[i] = t;
    zd[i] = (nz > 1 && in) ? 1.0 / (t_logz[j + 1] - t_logz[j]) : 0.0;
    zk[i] = k;
    zf[i] = f;
    mr[i] = mass[i] / (edges[i + 1] - edges[i]);
    gzeta[i] = 0.0;
  }
  int ja = 0;
  double ta = 0.0, dta = 0.0;
  if (nf > 1) {
    bool in;
    split_in_lds(t_afe, nf, th[TH_AFE], ja, ta, in);
    dta = in ? 1.0 / (t_afe[ja + 1] - t_afe[ja]) : 0.0;
  }
  __syncthreads();

  // ---- lines: recompute the young weights and Q-weighted sums, then back to W and gas
  double ggz = 0.0, ggu = 0.0;
  if (nl > 0) {
    for (int ag = tid; ag < ny; ag += 256) {   // young ages: first bin by bisection
      const double lo = s_clo[ag], hi = s_chi[ag];
      int i = 0;
      {
        int l = 0, h = n;
        while (l < h) {
          const int mid = (l + h) >> 1;
          if (edges[mid + 1] > lo) h = mid; else l = mid + 1;
        }
        i = l;
      }
      for (; i < n && edges[i] < hi; ++i) {
        const double ov = fmin(hi, edges[i + 1]) - fmax(lo, edges[i]);
        if (ov <= 0.0) continue;
        const double w = mr[i] * ov;
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
    }
    __syncthreads();
    {   // photon-weighted young mass per age: eight lanes per age, fixed butterfly
      const int nm = nf * nz;
      for (int g0 = 0; g0 < ny; g0 += 32) {
        const int ag = g0 + (tid >> 3), c = tid & 7;
        double sacc = 0.0;
        if (ag < ny)
          for (int q = c; q < nm; q += 8) {
            const int ia = q / nz, m = q - ia * nz;
            sacc += wrow[kpos_of(lib, ia, m, ag)] * s_Q[q * ny + ag];
          }
        sacc += __shfl_xor(sacc, 1);
        sacc += __shfl_xor(sacc, 2);
        sacc += __shfl_xor(sacc, 4);
        if (ag < ny && c == 0) wq[ag] = sacc;
      }
    }
    __syncthreads();
    int jg = 0, ju = 0;
    double tg = 0.0, tu = 0.0;
    bool ig, iu;
    split_in_lds(s_zg, lib.n_zg, th[TH_GAS_LOGZ], jg, tg, ig);
    split_in_lds(s_un, lib.n_u, th[TH_GAS_LOGU], ju, tu, iu);
    const double dtg = ig ? 1.0 / (s_zg[jg + 1] - s_zg[jg]) : 0.0;
    const double dtu = iu ? 1.0 / (s_un[ju + 1] - s_un[ju]) : 0.0;
    const int nu = lib.n_u;
    const size_t slab = (size_t)nl * ny;
    const double *t00p = lib.line_table + (size_t)(jg * nu + ju) * slab;
    const double *t01p = lib.line_table + (size_t)(jg * nu + ju + 1) * slab;
    const double *t10p = lib.line_table + (size_t)((jg + 1) * nu + ju) * slab;
    const double *t11p = lib.line_table + (size_t)((jg + 1) * nu + ju + 1) * slab;
    const double c00 = (1 - tg) * (1 - tu), c01 = (1 - tg) * tu, c10 = tg * (1 - tu), c11 = tg * tu;
    // thread (line group g = tid / 32, age slot tid % 32): the lines l = g, g + 8, ...;
    // 10^Lhat and its gas derivatives per (line, age), four lines' table loads in flight
    if (a.f64) {
    for (int a0 = 0; a0 < ny; a0 += 32) {
      const int ag = a0 + (tid & 31), g = tid >> 5;
      const bool act = ag < ny;
      const int agc = act ? ag : 0;
      const double wq_a = wq[agc];
      double gs = 0.0;
      for (int l0 = g; l0 < nl; l0 += 32) {
        double v[4][4], gLv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int l = min(l0 + 8 * u, nl - 1);
          const size_t q = (size_t)l * ny + agc;
          v[u][0] = t00p[q];
          v[u][1] = t01p[q];
          v[u][2] = t10p[q];
          v[u][3] = t11p[q];
          gLv[u] = pr.kind == 0 ? gacc[a.line_k0 + l] / kLsun : a.dLl[(size_t)r * nl + l];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (!act || l0 + 8 * u >= nl) continue;
          const double lh = c00 * v[u][0] + c01 * v[u][1] + c10 * v[u][2] + c11 * v[u][3];
          const double E = exp10(lh);
          gs += gLv[u] * E;
          const double gE = gLv[u] * wq_a * E * 2.302585092994046;
          ggz += gE * ((1 - tu) * (v[u][2] - v[u][0]) + tu * (v[u][3] - v[u][1])) * dtg;
          ggu += gE * ((1 - tg) * (v[u][1] - v[u][0]) + tg * (v[u][3] - v[u][2])) * dtu;
        }
      }
      if (act) red[g * ny + ag] = gs;
    }
    } else {
    // FP32 gradient pass: the FP32 table and exponentials (the result feeds FP32 weights)
    const size_t slab_f = (size_t)nl * ny;
    const float *f00p = lib.line_table_f + (size_t)(jg * nu + ju) * slab_f;
    const float *f01p = lib.line_table_f + (size_t)(jg * nu + ju + 1) * slab_f;
    const float *f10p = lib.line_table_f + (size_t)((jg + 1) * nu + ju) * slab_f;
    const float *f11p = lib.line_table_f + (size_t)((jg + 1) * nu + ju + 1) * slab_f;
    const float e00 = (float)c00, e01 = (float)c01, e10 = (float)c10, e11 = (float)c11;
    for (int a0 = 0; a0 < ny; a0 += 32) {
      const int ag = a0 + (tid & 31), g = tid >> 5;
      const bool act = ag < ny;
      const int agc = act ? ag : 0;
      const double wq_a = wq[agc];
      double gs = 0.0;
      for (int l0 = g; l0 < nl; l0 += 64) {
        float v[8][4];
        double gLv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int l = min(l0 + 8 * u, nl - 1);
          const size_t q = (size_t)l * ny + agc;
          v[u][0] = f00p[q];
          v[u][1] = f01p[q];
          v[u][2] = f10p[q];
          v[u][3] = f11p[q];
          gLv[u] = pr.kind == 0 ? gacc[a.line_k0 + l] / kLsun : a.dLl[(size_t)r * nl + l];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (!act || l0 + 8 * u >= nl) continue;
          const float lh = e00 * v[u][0] + e01 * v[u][1] + e10 * v[u][2] + e11 * v[u][3];
          const double E = (double)exp10f(lh);
          gs += gLv[u] * E;
          const double gE = gLv[u] * wq_a * E * 2.302585092994046;
          ggz += gE * (double)((1.f - (float)tu) * (v[u][2] - v[u][0]) + (float)tu * (v[u][3] - v[u][1])) * dtg;
          ggu += gE * (double)((1.f - (float)tg) * (v[u][1] - v[u][0]) + (float)tg * (v[u][3] - v[u][2])) * dtu;
        }
      }
      if (act) red[g * ny + ag] = gs;
    }
    }
    __syncthreads();
    for (int ag = tid; ag < ny; ag += 256) {   // the eight line groups in a fixed order
      double gs = 0.0;
      for (int g = 0; g < 8; ++g) gs += red[g * ny + ag];
      gwq[ag] = gs;
    }
    __syncthreads();
    for (int e = tid; e < ny * nz * nf; e += 256) {   // young entries (age, alpha, Z)
      const int ag = e / (nz * nf), q = e - ag * (nz * nf), ia = q / nz, m = q - ia * nz;
      gacc[kpos_of(lib, ia, m, ag)] += gwq[ag] * s_Q[(ia * nz + m) * ny + ag];
    }
    __syncthreads();
  }

  // ---- weights adjoint: thread per SFH bin, ages in increasing order
  double gz_e = 0.0, gafe = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double Ti = edges[i], Tj = edges[i + 1], dTb = Tj - Ti;
    const double inv = 1.0 / dTb, mri = mr[i];
    int ag;
    {
      int l = 0, h = na;   // first cell whose upper edge exceeds Ti
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (s_chi[mid] > Ti) h = mid; else l = mid + 1;
      }
      ag = l;
    }
    double gmi = 0.0, gzi = 0.0;
    const int j0 = zj[i];
    const double t0 = zt[i], zdi = zd[i];
    for (; ag < na && s_clo[ag] < Tj; ++ag) {
      const double lo = s_clo[ag], hi = s_chi[ag];
      const double upper = fmin(hi, Tj), lower = fmax(lo, Ti);
      const double ovr = upper - lower;
      if (ovr <= 0.0) continue;
      const double w = mri * ovr;
      double gw = 0.0;
      for (int q = 0; q < (nf > 1 ? 2 : 1); ++q) {
        const int ia = nf > 1 ? ja + q : 0;
        const double fa = nf > 1 ? (q == 0 ? 1.0 - ta : ta) : 1.0;
        const double dfa = nf > 1 ? (q == 0 ? -dta : dta) : 0.0;
        double gA;
        if (nz > 1) {
          const double g0 = gacc[kpos_of(lib, ia, j0, ag)];
          const double g1 = gacc[kpos_of(lib, ia, j0 + 1, ag)];
          gA = (1.0 - t0) * g0 + t0 * g1;
          gzi += fa * zdi * w * (g1 - g0);
        } else {
          gA = gacc[kpos_of(lib, ia, 0, ag)];
        }
        gw += fa * gA;
        gafe += dfa * w * gA;
      }
      gmi += gw * ovr * inv;
      // w = m ov / dT with ov = min(hi, T_j) - max(lo, T_i): its edge derivatives
      const double dov_i = (Ti > lo) ? -1.0 : 0.0;
      const double dov_j = (Tj < hi) ? 1.0 : 0.0;
      const double dw_i = mri * (dov_i + ovr * inv);
      const double dw_j = mri * (dov_j - ovr * inv);
      gz_e += gw * (dw_i * dT[i] + dw_j * dT[i + 1]);
    }
    gr[TH_NSCALAR + i] = gmi;   // d logL / d m_i
    gzeta[i] = gzi;
  }
  // four block sums at once: wave butterflies, then the four waves in a fixed order
  double v4[4] = {gz_e, gafe, ggz, ggu};
#pragma unroll
  for (int k = 0; k < 4; ++k)
    for (int o = 32; o > 0; o >>= 1) v4[k] += __shfl_xor(v4[k], o, 64);
  __syncthreads();
  if ((tid & 63) == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[(tid >> 6) * 4 + k] = v4[k];
  __syncthreads();
  const double s_ze = (red[0] + red[4]) + (red[8] + red[12]), s_afe = (red[1] + red[5]) + (red[9] + red[13]);
  const double s_gz = (red[2] + red[6]) + (red[10] + red[14]), s_gu = (red[3] + red[7]) + (red[11] + red[15]);
  const double *gb = a.gbuf + (size_t)r * 16;
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
    if (lib.n_zh == 0) {   // constant metallicity: every bin's share, in bin order
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += gzeta[i];
      gr[TH_LOGZSOL] = s;
    }
  }
  // metallicity-history nodes: transpose of the bin interpolation, one thread per node,
  // each adding its bins' shares in bin order (bin 0 takes node 0 alone).  The node
  // index of bins 1..n-1 does not decrease with the bin, so node k's bins (index k - 1
  // or k) are one run, found by bisection.
  if (lib.n_zh > 0)
    for (int k = tid; k < lib.n_zh; k += 256) {
      double sk = k == 0 ? gzeta[0] : 0.0;
      int l = 1, h = n;   // first bin >= 1 whose node index reaches k - 1
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (zk[mid] < k - 1) l = mid + 1; else h = mid;
      }
      for (int i = l; i < n && zk[i] <= k; ++i) {
        if (zk[i] == k) sk += (1.0 - zf[i]) * gzeta[i];
        else sk += zf[i] * gzeta[i];   // zk[i] == k - 1
      }
      gr[TH_NSCALAR + n + k] = sk;
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
  aa.f_spans = w.f_spans && g.log_uniform ? 1 : 0;
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
  // dynamic LDS of the projection adjoint: gF [N] in the pass's precision (FP32 spectra:
  // the span of the rows), the line tables of a spectrum, then on the FP32 path the
  // per-node or per-pixel tables of the transpose when they fit (two workgroups per CU)
  const bool spec = o->host.kind != 0;
  size_t gb = ((size_t)g.N * 8 + 15) & ~(size_t)15, extra = 0;
  aa.fast = 0;
  aa.seg_cap = 0;
  aa.nl_lds = spec ? g.n_line : 0;
  const size_t lines_b = 40 * (size_t)aa.nl_lds;
  if (!f64 && !spec && g.log_uniform) {
    const size_t nfn = o->host.fw.size(), nb = o->host.band_off.size();
    const size_t t = 4 * nb + 16;
    if (gb + t <= 76 * 1024) {
      extra = t;
      aa.fast = 1;
    }
  } else if (!f64 && spec && g.log_uniform && o->host.n_data > 0) {
    const size_t np = (size_t)o->host.n_data;
    double kmax = 0.0;
    for (double v : o->host.ksig) kmax = std::max(kmax, v);
    // the longest span spec_span gives a row at any redshift, plus the rounding of its ends
    const double span = (o->host.lnpix.back() - o->host.lnpix.front()) * g.inv_dlnw + 2.0 * spec_span_ext(kmax, g.inv_dlnw);
    const size_t cap = (size_t)std::min((double)g.N, std::ceil(span) + 4.0);
    const size_t gbf = (cap * 4 + 15) & ~(size_t)15;
    const size_t t = ((4 * np + 15) & ~(size_t)15) + 12 * np + 2048 + 8 * (np / 16 + 2);
    if (gbf + lines_b + t <= 76 * 1024 && cap <= 256 * (size_t)kAdjOwn) {
      gb = gbf;
      extra = t;
      aa.fast = 1;
      aa.seg_cap = (int)cap;
    }
  }
  aa.g_bytes = (int)gb;
  aa.fr_max = 0.0;
  for (double v : o->host.fr) aa.fr_max = std::max(aa.fr_max, std::fabs(v));

  const size_t sm1 = gb + lines_b + extra;
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
  int n_split = 1;   // FP32 dW: wavelength halves (see below)
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    if (f64) {
      hipLaunchKernelGGL(k_bwd_f64, dim3((B_pad / 64) * (g.K_pad / 64)), dim3(256), 0, s, (const double *)aa.GY,
                         (const double *)aa.GO, g.LT64, g.N_pad, g.K_pad, g.K_young_pad, (double *)w.dW);
    } else {
      // halve the wavelength range over two blocks per output tile when that lowers the
      // largest number of tiles any CU has to finish (four blocks fit a CU)
      const int n_tiles = (B_pad / 64) * (g.K_pad / 64);
      const int full = (n_tiles + 255) / 256, halves = (2 * n_tiles + 255) / 256;
      n_split = halves < 2 * full ? 2 : 1;
      hipLaunchKernelGGL((k_bwd_f32<64, 64>), dim3(n_tiles * n_split), dim3(256), 0, s, (const float *)aa.GY,
                         (const float *)aa.GO, g.L32n, g.N_pad, g.K_pad, g.K_young_pad, (const uint32_t *)w.rowmask,
                         w.mask_words, (double *)w.dW, n_split, (size_t)w.B_pad_max * g.K_pad,
                         g.log_uniform ? (const PointRow *)w.rows : nullptr);
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
    ap.dW2 = n_split == 2 ? (const double *)w.dW + (size_t)w.B_pad_max * g.K_pad : nullptr;
    ap.f64 = f64 ? 1 : 0;
    ap.kpos = L->kpos_d;
    ap.line_k0 = L->line_k0;
    ap.gbuf = w.gbuf;
    ap.gnoise = w.gnoise;
    ap.dLl = w.dLl;
    ap.grad = grad;
    const size_t sm2 = sizeof(double) * (size_t)AdjPrepSmem(g).total;
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
