// Observer-frame projection (Sec. 2.6, App. E, App. F) and the diagonal Gaussian
// log-likelihood with the noise floor (eq. 6, eq. G1).  One workgroup per sorted
// row; the chi-squared sum is accumulated in FP64 and reduced in a fixed order.
#include "common.h"
#include "kernels.h"

namespace sps {

constexpr int kLineCut = 10;   // analytic line profiles evaluated within 10 sigma
constexpr int kLineCatMax = 256;   // entries of a catalogue marginalised jointly with a spectrum

template <typename T>
struct ProjArgs {
  const DevObs *obs_table;
  const PointRow *rows;
  const T *F;
  int N_pad, n_line;
  const double *theta;
  int P, B;
  const double *Lline;
  double *model, *logl, *gvec, *gnoise, *msorted;
  int ld_model, ld_g;
};

__device__ __forceinline__ double wave_reduce_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sigma_inst(lambda_obs) in km/s for an LSF mode (eq. F2); `v` is the constant
// or the curve value interpolated at lambda.
__device__ double sigma_inst_mode(int mode, double v, double lam) {
  switch (mode) {
    case 0: return kC_kms / (2.3548200450309493 * v);   // R_fwhm
    case 1: return kC_kms / v;                          // R_sigma
    case 2: return kC_kms * v / (2.3548200450309493 * lam);
    case 3: return kC_kms * v / lam;
    case 4: return v;
    default: return v / 2.3548200450309493;
  }
}

// The IGM transmission where the kernel was built with it (IGM = lib.igm), else 1: a
// template argument so that kernels without the IGM do not carry its registers.
template <bool IGM>
__device__ __forceinline__ double igm_at(const DevLib &lib, const double *th, double z, double lam) {
  if constexpr (IGM) return igm_T(lib, th, z, lam);
  else return 1.0;
}

// A library line at one point of a spectrum (App. I.1, eq. app_line_profile): its observer-
// frame flux (the young light's birth-cloud transmission with an escape geometry's mixture,
// the diffuse screen, mass over 4 pi D_L^2 and the IGM at the line), its observed wavelength
// and its profile width in ln(lambda) (gas dispersion and the instrument at the line).
template <bool IGM>
__device__ __forceinline__ void spec_line_terms(const DevLib &lib, const DevObs &ob, const PointRow &pr,
                                                const double *th, double Lline, int l, double &Fl, double &lobs,
                                                double &sl) {
  const double z = pr.z, opz = 1.0 + z;
  const double Tfac = pr.mass10 / (4.0 * kPi * pr.dl * pr.dl);
  const double lw = lib.line_wave[l];
  const double lnlv = log(lw / kLamV);
  const double tbc = pr.bc_p * exp(-pr.tau_bc * exp(pr.alpha_bc * lnlv)) + pr.bc_q;
  const double td = exp(-pr.tau_diff * exp(pr.delta * lnlv) * (lib.line_a[l] + (0.85 - 1.9 * pr.delta) * lib.line_d[l]));
  lobs = opz * lw;
  Fl = Lline * tbc * td * Tfac * igm_at<IGM>(lib, th, z, lobs);
  double v = ob.lsf_value;
  if (ob.has_curve) {
    const int np = ob.n_data;
    const double lc = fmin(fmax(lobs, ob.pix[0]), ob.pix[np - 1]);
    const int k = bracket(ob.pix, np, lc);
    const double t = (lc - ob.pix[k]) / (ob.pix[k + 1] - ob.pix[k]);
    v = ob.lsf_vals[k] + t * (ob.lsf_vals[k + 1] - ob.lsf_vals[k]);
  }
  const double si = sigma_inst_mode(ob.lsf_mode, v, lobs);
  sl = sqrt(ob.sigma_gas_kms * ob.sigma_gas_kms + si * si) / kC_kms;
}

template <typename T, bool IGM>
__global__ void __launch_bounds__(256, IGM ? 3 : 4) k_project(DevLib lib, ProjArgs<T> a) {
  __shared__ double red[256];
  // LDS: per-line tables (spectra) and, on the FP32 path, a segment of the model row
  // (photometry: the pixels under the filters; spectra: the pixels under the LSF rows);
  // the generic photometry path keeps per-node terms instead
  constexpr int kLineBytes = 3 * 512 * 8, kTermBytes = 4096 * (int)sizeof(T);
  constexpr int kSegOff = kLineBytes, kSegMax = sizeof(T) == 4 ? 4096 : 0;
  constexpr int kRaw1 = kSegOff + 4 * kSegMax;
  constexpr int kRaw = kRaw1 > kTermBytes ? kRaw1 : kTermBytes;
  constexpr int kClBytes = sizeof(T) == 4 ? 512 * 4 : 0;   // FP32 spectra: per-line exponent factors
  __shared__ __attribute__((aligned(16))) unsigned char sraw[kRaw + kClBytes];
  T *s_term = (T *)sraw;
  double *s_lnl = (double *)sraw, *s_isl = s_lnl + 512, *s_amp = s_lnl + 1024;
  float *s_cl = (float *)(sraw + kRaw);
  __shared__ double s_slmax[4];
  const int r = blockIdx.x;
  const PointRow pr = a.rows[r];
  if (pr.b < 0) return;
  const int tid = threadIdx.x;
  const T *Fr = a.F + (size_t)r * a.N_pad;
  const int N = lib.N;
  // FP32 photometry on a log-uniform rest grid: the model pixels under the filters (the
  // rest-frame span of the nodes, from the weight builder) are requested first, before
  // the observation's descriptor is read, sixteen loads per thread in flight
  const bool fastp = sizeof(T) == 4 && lib.log_uniform && !a.gvec && pr.kind == 0 && pr.seg_n <= kSegMax;
  if (fastp) {
    float *seg = (float *)(sraw + kSegOff);
    const int seg0 = pr.seg0, seg_n = pr.seg_n;
    for (int k0 = tid; k0 < seg_n; k0 += 256 * 16) {
      float v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = (float)Fr[seg0 + min(k0 + 256 * q, seg_n - 1)];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (k0 + 256 * q < seg_n) seg[k0 + 256 * q] = v[q];
    }
    if (IGM) {   // the IGM transmission at lambda (1 + z) of the pixels blueward of Ly alpha (FP64:
                     // optical depths of tens amplify FP32 rounding past the FP32 tolerance)
      const double *thb = a.theta + (size_t)pr.b * a.P;
      for (int k = tid; k < seg_n; k += 256) seg[k] *= (float)igm_at<IGM>(lib, thb, pr.z, lib.wave_d[seg0 + k] * (1.0 + pr.z));
    }
  }
  const DevObs ob = a.obs_table[pr.obs];
  const double *th = a.theta + (size_t)pr.b * a.P;
  const double z = pr.z, opz = 1.0 + z;

  // noise-floor parameters (ln space), evaluated by every thread (no barrier)
  const double ns = (ob.noise_flags & 1) ? exp(th[TH_LOG_ERR_SCALE]) : 1.0;
  const double fc = (ob.noise_flags & 2) ? exp(th[TH_LOG_F_CALIB]) : 0.0;
  const double fd = (ob.noise_flags & 4) ? exp(th[TH_LOG_F_DATA]) : 0.0;
  const double jt = (ob.noise_flags & 8) ? exp(th[TH_LOG_JITTER]) : 0.0;
  double lsum = 0.0;
  double gs[4] = {0.0, 0.0, 0.0, 0.0};

  auto datum_in = [&](int i, double m, bool mk, double d, double sg) {
    if (a.model) a.model[(size_t)pr.b * a.ld_model + i] = m;
    if (a.msorted) a.msorted[(size_t)r * a.ld_g + i] = m;
    double g = 0.0;
    if (mk) {
      const double v = ns * ns * sg * sg + fc * fc * m * m + fd * fd * d * d + jt * jt;
      const double res = d - m;
      lsum += -0.5 * res * res / v - 0.5 * log(2.0 * kPi * v);
      // d logL / d v and d logL / d m (App. G terms)
      const double dv = 0.5 * res * res / (v * v) - 0.5 / v;
      g = res / v + dv * 2.0 * fc * fc * m;
      if (ob.noise_flags & 1) gs[0] += dv * 2.0 * ns * ns * sg * sg;   // d/d ln s
      gs[1] += dv * 2.0 * fc * fc * m * m;     // d/d ln f_calib
      gs[2] += dv * 2.0 * fd * fd * d * d;     // d/d ln f_data
      gs[3] += dv * 2.0 * jt * jt;             // d/d ln j
    }
    if (a.gvec) a.gvec[(size_t)r * a.ld_g + i] = g;
  };
  auto datum = [&](int i, double m) { datum_in(i, m, ob.mask[i] != 0, ob.data[i], ob.sigma[i]); };

  if (ob.kind == 0) {
    // ---------------- photometry (eq. E1-E2): f_lambda^obs(lambda_j) = fac * F(lambda_j/(1+z))
    const double fac = kC_cms * pr.scale_fnu / (opz * opz * kAng_cm * kAng_cm);
    const double lnopz = log1p(z);
    const double wlo = lib.wave_d[0], whi = lib.wave_d[N - 1];
    // On a log-uniform rest grid the bracketing interval follows from ln(lambda)
    // directly; a node within rounding of a grid point may take the neighbouring
    // interval, where the interpolation weight is within rounding of 0 or 1.
    // FP32 path (fastp): each wave takes whole bands, lanes over the band's nodes, and
    // reduces them itself.  The weight linear in lambda on [w_k, w_k+1] is
    // (e^{f d} - 1)/(e^d - 1), f the fractional log index; a node is inside the model grid
    // when its log index lies in [0, N - 1].
    // (the gradient pass keeps the generic path: its band sums are accumulated in FP64)
    if (fastp) {
      const float *seg = (const float *)(sraw + kSegOff);
      const int seg0 = pr.seg0, seg_n = pr.seg_n;
      // this thread's band datum, requested before the band sums
      const int bi = min(tid, ob.n_band - 1);
      const double d_b = ob.data[bi], s_b = ob.sigma[bi];
      const bool m_b = ob.mask[bi] != 0;
      const double ui0 = phot_ui0(lib, z);
      const double d = 1.0 / lib.inv_dlnw;
      const float df = (float)d, inv_em1 = (float)(1.0 / expm1(d));
      // e^x - 1 for x = f d in [0, d]: below d = 0.05 the series to x^4 is exact to FP32
      // rounding (and free of the cancellation of expf(x) - 1)
      const bool series = d < 0.05;
      const double umax = (double)(N - 1);
      // the wave index made explicitly uniform, so that the band offsets are scalar loads
      const int wave_id = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
      __syncthreads();
      // wave w takes bands w, w+4, ..., eight at a time, so that all their node loads are
      // in flight together (issued unconditionally from clamped indices) and their eight
      // wave reductions interleave
      for (int g0 = wave_id; g0 < ob.n_band; g0 += 32) {
        float part[8];
        int jlo[8], jhi[8], len = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int band = g0 + 4 * i, bc = min(band, ob.n_band - 1);
          const int lo = ob.band_off[bc], hi = ob.band_off[bc + 1];
          jlo[i] = band < ob.n_band ? lo : 0;
          jhi[i] = band < ob.n_band ? hi : 0;
          len = max(len, jhi[i] - jlo[i]);
          part[i] = 0.f;
        }
        for (int jb = 0; jb < len; jb += 128) {   // two nodes per lane and band per pass
          double uq[16];
          float rq[16];
          bool ok[16];
#pragma unroll
          for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int j = jlo[i] + jb + 64 * q + lane;
              ok[2 * i + q] = j < jhi[i];
              const int jc = j < jhi[i] ? j : 0;
              uq[2 * i + q] = ob.fwln[jc];
              rq[2 * i + q] = ob.fr_f[jc];
            }
#pragma unroll
          for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int n = 2 * i + q;
              const double u = phot_u(lib, uq[n], ui0);
              const bool in = ok[n] && u >= 0.0 && u <= umax;
              const int k = min(max((int)floor(u), 0), N - 2);
              const int kk = in ? min(max(k - seg0, 0), seg_n - 2) : 0;
              const float x = (float)(u - (double)k) * df;
              float em;
              if (series) em = x * (1.f + x * (0.5f + x * (1.f / 6.f + x * (1.f / 24.f))));
              else em = expf(x) - 1.f;
              const float t = em * inv_em1;
              const float f0 = seg[kk], f1 = seg[kk + 1];
              part[i] += in ? rq[n] * (f0 + t * (f1 - f0)) : 0.f;
            }
        }
        // FP32 butterfly (the terms are FP32 products; at most 4096 of them per band)
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
          for (int i = 0; i < 8; ++i) part[i] += __shfl_xor(part[i], o, 64);
        }
        if (lane == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (g0 + 4 * i < ob.n_band) red[g0 + 4 * i] = (double)part[i];
        }
      }
      __syncthreads();
      if (tid < ob.n_band) datum_in(tid, fac * red[tid], m_b, d_b, s_b);   // n_band <= 256
    } else {
      // one pass over all filter nodes, eight per thread in flight, terms kept in LDS
      for (int j0 = tid; j0 < ob.n_fnodes; j0 += 2048) {
        int kq[8];
        double lrq[8];
        bool in[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = j0 + 256 * q;
          in[q] = false;
          kq[q] = 0;
          lrq[q] = 0.0;
          if (j < ob.n_fnodes) {
            lrq[q] = ob.fw[j] / opz;
            in[q] = lrq[q] >= wlo && lrq[q] <= whi;
            if (in[q]) {
              if (lib.log_uniform) {
                const int k = (int)floor((ob.fwln[j] - lnopz - lib.lnw0) * lib.inv_dlnw);
                kq[q] = min(max(k, 0), N - 2);
              } else {
                kq[q] = bracket(lib.wave_d, N, lrq[q]);
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = j0 + 256 * q;
          if (j < ob.n_fnodes) {
            double term = 0.0;
            if (in[q]) {
              const int k = kq[q];
              const double w0 = lib.wave_d[k], w1 = lib.wave_d[k + 1];
              const T f0 = Fr[k] * (T)igm_at<IGM>(lib, th, z, w0 * opz), f1 = Fr[k + 1] * (T)igm_at<IGM>(lib, th, z, w1 * opz);
              const T w = sizeof(T) == 8 ? (T)ob.fr_d[j] : (T)ob.fr_f[j];
              const T t = (T)((lrq[q] - w0) / (w1 - w0));
              term = (double)(w * (f0 + t * (f1 - f0)));
            }
            s_term[j] = (T)term;
          }
        }
      }
      __syncthreads();
      // fixed-order band sums: one wave per band
      const int wave_id = tid >> 6, lane = tid & 63;
      for (int band = wave_id; band < ob.n_band; band += 4) {
        const int j0 = ob.band_off[band], j1 = ob.band_off[band + 1];
        double part = 0.0;
        for (int j = j0 + lane; j < j1; j += 64) part += (double)s_term[j];
        const double s = wave_reduce_sum(part);
        if (lane == 0) red[band] = s;
      }
      __syncthreads();
      for (int band = tid; band < ob.n_band; band += 256) datum(band, fac * red[band]);
    }
  } else if (ob.kind == 2) {
    // ---------------- emission-line catalogue (App. I.1-I.2): the line fluxes through the
    // young light's birth-cloud transmission, the diffuse screen, mass over 4 pi D_L^2 and
    // the IGM at the line, summed over each entry's blend; detections take the Gaussian
    // chi-squared, upper limits its one-sided form, logL = -chi^2 / 2 (no normalisation)
    double *s_fl = s_lnl;   // [n_line] line fluxes, erg/s/cm^2
    const int nl = a.n_line;
    const double Tfac = pr.mass10 / (4.0 * kPi * pr.dl * pr.dl);
    for (int l = tid; l < nl; l += 256) {
      const double lw = lib.line_wave[l];
      const double lnlv = log(lw / kLamV);
      const double tbc = pr.bc_p * exp(-pr.tau_bc * exp(pr.alpha_bc * lnlv)) + pr.bc_q;
      const double td = exp(-pr.tau_diff * exp(pr.delta * lnlv) * (lib.line_a[l] + (0.85 - 1.9 * pr.delta) * lib.line_d[l]));
      s_fl[l] = a.Lline[(size_t)r * nl + l] * tbc * td * Tfac * igm_at<IGM>(lib, th, z, opz * lw);
    }
    __syncthreads();
    for (int k = tid; k < ob.n_data; k += 256) {
      double m = 0.0;
      for (int j = ob.loff[k]; j < ob.loff[k + 1]; ++j) m += s_fl[ob.lidx[j]];
      if (a.model) a.model[(size_t)pr.b * a.ld_model + k] = m;
      if (a.msorted) a.msorted[(size_t)r * a.ld_g + k] = m;
      if (ob.mask[k]) {
        const double res = (ob.data[k] - m) / ob.sigma[k];
        if (!ob.upper[k] || m > ob.data[k]) lsum -= 0.5 * res * res;
      }
    }
  } else {
    // ---------------- spectrum (eq. F5-F6)
    const double lnopz = log1p(z);
    const int nl = a.n_line;
    double slmax = 0.0;
    if (nl > 0) {
      double my_max = 0.0;
      for (int l = tid; l < nl; l += 256) {
        double Fl, lobs, sl;
        spec_line_terms<IGM>(lib, ob, pr, th, a.Lline[(size_t)r * nl + l], l, Fl, lobs, sl);
        s_lnl[l] = log(lobs);
        s_isl[l] = 1.0 / sl;
        s_amp[l] = Fl / (2.5066282746310002 * sl);
        if (sizeof(T) == 4) s_cl[l] = (float)(-0.72134752044448170 / (sl * sl));   // -log2(e) / (2 sl^2)
        my_max = fmax(my_max, sl);
      }
      for (int o = 32; o > 0; o >>= 1) my_max = fmax(my_max, __shfl_xor(my_max, o, 64));
      if ((tid & 63) == 0) s_slmax[tid >> 6] = my_max;
      __syncthreads();
      slmax = fmax(fmax(s_slmax[0], s_slmax[1]), fmax(s_slmax[2], s_slmax[3]));
    }
    const double lnw0 = lib.lnwave_d[0], lnw1 = lib.lnwave_d[N - 1];
    // FP32 path on a log-uniform rest grid: the rows' span of model pixels, times
    // lambda^2, is staged in LDS; the Gaussian row weights come from the recurrence
    // w_{j+1} = w_j q_j, q_{j+1} = q_j e^{-h^2} (h = node spacing / row width), which
    // needs three exponentials per row instead of one per tap
    int seg0 = 0, seg_n = 0;
    const bool fast = sizeof(T) == 4 && lib.log_uniform;   // the adjoint transposes the same rows
    if (fast) spec_span(lib, ob.lnpix_lo, ob.lnpix_hi, ob.ksig_max, z, seg0, seg_n);
    if (fast && seg_n <= kSegMax) {
      float *seg = (float *)(sraw + kSegOff);
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
      if (IGM)   // the IGM transmission at lambda (1 + z), blueward of Ly alpha (FP64), on the
                 // entries this thread staged
        for (int k = tid; k < seg_n; k += 256) seg[k] *= (float)igm_at<IGM>(lib, th, z, lib.wave_d[seg0 + k] * opz);
      __syncthreads();
      const double dln = 1.0 / lib.inv_dlnw;
      int lwin = 0;   // start of the line window: pixels rise with i, so it only moves up
      // the next pixel's inputs are loaded while the current one is computed
      struct PixIn {
        double lnp, ks, px, d, sg, iv;
        bool mk;
      };
      // no noise-floor terms and no adjoint outputs: the constant-noise form of eq. 6
      const bool const_noise = ob.noise_flags == 0 && !a.gvec && !a.gnoise && !a.msorted;
      auto pix_in = [&](int i) {
        PixIn v;
        const int ic = i < ob.n_data ? i : 0;
        v.lnp = ob.lnpix[ic];
        v.ks = ob.ksig[ic];
        v.px = ob.pix[ic];
        v.d = ob.data[ic];
        v.sg = ob.sigma[ic];
        v.iv = ob.ivar[ic];
        v.mk = ob.mask[ic] != 0;
        return v;
      };
      PixIn nxt = pix_in(tid);
      for (int i = tid; i < ob.n_data; i += 256) {
        const PixIn cur = nxt;
        nxt = pix_in(i + 256);
        const double x = cur.lnp - lnopz;
        float cont = 0.f;
        if (x >= lnw0 && x <= lnw1) {
          const double s = cur.ks;
          const double ux = (x - lnw0) * lib.inv_dlnw;   // fractional node index of x
          if (s < 0.5 * dln) {
            const int k = min((int)floor(ux), N - 2);
            const float t = (float)(ux - (double)k);
            const float g0 = seg[k - seg0], g1 = seg[k + 1 - seg0];
            cont = g0 + t * (g1 - g0);
          } else {
            const double rs = s * lib.inv_dlnw;            // row width in node spacings
            const int j0 = max((int)ceil(ux - 5.0 * rs), 0);
            const int j1 = min((int)floor(ux + 5.0 * rs), N - 1);
            const float h = 1.f / (float)rs, a0 = (float)((double)j0 - ux) * h;
            float w = expf(-0.5f * a0 * a0);
            float q = expf(-a0 * h - 0.5f * h * h);
            const float c = expf(-h * h);
            // eight taps per step: their LDS reads are independent of the recurrence, and
            // every step restarts it from the exact Gaussian (two exponentials), so that
            // the FP32 rounding of q and c compounds over at most eight taps however wide
            // the row (a row of a few hundred taps drifted by ~1e-5 otherwise)
            float num = 0.f, den = 0.f;
            const float *gp = seg + (j0 - seg0);
            const int nt = j1 - j0 + 1;
            int jj = 0;
            for (; jj + 8 <= nt; jj += 8) {
              float g[8];
#pragma unroll
              for (int e = 0; e < 8; ++e) g[e] = gp[jj + e];
              if (jj > 0) {
                const float a = a0 + (float)jj * h;
                w = expf(-0.5f * a * a);
                q = expf(-a * h - 0.5f * h * h);
              }
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                num += w * g[e];
                den += w;
                w *= q;
                q *= c;
              }
            }
            for (; jj < nt; ++jj) {
              num += w * gp[jj];
              den += w;
              w *= q;
              q *= c;
            }
            cont = num / den;
          }
        }
        double m = pr.scale_fnu * (double)cont;
        if (nl > 0) {
          const double lp = cur.lnp;
          while (lwin < nl && s_lnl[lwin] < lp - kLineCut * slmax) ++lwin;
          double lines = 0.0;
          // the Gaussian as 2^(d^2 c_l), d = ln(lambda) offset in FP32 (|d| <= 10 sigma), one
          // hardware exp2 per line; the amplitude and the sum stay FP64
          for (int l = lwin; l < nl && s_lnl[l] <= lp + kLineCut * slmax; ++l) {
            const float d = (float)(lp - s_lnl[l]);
            lines += s_amp[l] * (double)__builtin_amdgcn_exp2f(d * d * s_cl[l]);
          }
          m += lines * cur.px * kAng_cm / kC_cms;
        }
        if (const_noise) {   // -1/2 sum (d - m)^2 / sigma^2; the ln(2 pi sigma^2) sum is added once
          const double mm = m / kFnuAB;
          if (a.model) a.model[(size_t)pr.b * a.ld_model + i] = mm;
          const double res = cur.d - mm;
          lsum -= 0.5 * res * res * cur.iv;
        } else {
          datum_in(i, m / kFnuAB, cur.mk, cur.d, cur.sg);
        }
      }
      if (const_noise && tid == 0) lsum += ob.lnorm;
    } else {
      for (int i = tid; i < ob.n_data; i += 256) {
        const double x = ob.lnpix[i] - lnopz;
        T cont = (T)0;
        if (x >= lnw0 && x <= lnw1) {
          const double s = ob.ksig[i];
          const int k = lnwave_bracket(lib, x);
          const double dk = lib.lnwave_d[k + 1] - lib.lnwave_d[k];
          if (s < 0.5 * dk) {
            const T t = (T)((x - lib.lnwave_d[k]) / dk);
            const T fk = Fr[k] * (T)(lib.lam2_d[k] * igm_at<IGM>(lib, th, z, lib.wave_d[k] * opz));
            const T fk1 = Fr[k + 1] * (T)(lib.lam2_d[k + 1] * igm_at<IGM>(lib, th, z, lib.wave_d[k + 1] * opz));
            cont = fk + t * (fk1 - fk);
          } else {
            int j = lnwave_lower_bound(lib, x - 5.0 * s);
            const double inv = 1.0 / s;
            double num = 0.0, den = 0.0;
            for (; j < N; ++j) {
              const double u = (lib.lnwave_d[j] - x) * inv;
              if (u > 5.0) break;
              const T w = sizeof(T) == 8 ? (T)exp(-0.5 * u * u) : (T)expf((float)(-0.5 * u * u));
              num += (double)(w * (Fr[j] * (T)(lib.lam2_d[j] * igm_at<IGM>(lib, th, z, lib.wave_d[j] * opz))));
              den += (double)w;
            }
            cont = (T)(num / den);
          }
        }
        double m = pr.scale_fnu * (double)cont;
        if (nl > 0) {
          const double lp = ob.lnpix[i];
          // lines sorted by wavelength: window of ln(lambda_obs) within kLineCut * s_max
          int l = lower_bound_dev(s_lnl, nl, lp - kLineCut * slmax);
          double lines = 0.0;
          for (; l < nl && s_lnl[l] <= lp + kLineCut * slmax; ++l) {
            const double u = (lp - s_lnl[l]) * s_isl[l];
            lines += s_amp[l] * exp(-0.5 * u * u);
          }
          m += lines * ob.pix[i] * kAng_cm / kC_cms;
        }
        datum(i, m / kFnuAB);
      }
    }
  }
  // fixed-order reduction of logL (and the noise-parameter gradients): wave sums,
  // then the four waves in order
  {
    const int wv = tid >> 6, lane = tid & 63;
    const double ws = wave_reduce_sum(lsum);
    double wg[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.gnoise)
      for (int q = 0; q < 4; ++q) wg[q] = wave_reduce_sum(gs[q]);
    __syncthreads();   // red[] may still be read by the band sums
    if (lane == 0) {
      red[wv] = ws;
      for (int q = 0; q < 4; ++q) red[4 + 4 * q + wv] = wg[q];
    }
    __syncthreads();
    if (tid == 0 && a.logl) a.logl[pr.b] = (red[0] + red[1]) + (red[2] + red[3]);
    if (a.gnoise && tid < 4) {
      const double *g = red + 4 + 4 * tid;
      a.gnoise[(size_t)pr.b * 4 + tid] = (g[0] + g[1]) + (g[2] + g[3]);
    }
  }
}

// ---------------------------------------------------------------------------------
// Spectrophotometric calibration polynomial (Sec. 3.2, App. H.3, eq. app_polymarg).  One
// workgroup per sorted row: with D = diag(mu) A (A_im = T_m(x_i), Chebyshev), C the noise
// of the uncalibrated model mu and r = d - mu over the mask, G = D^T C^-1 D and
// b = D^T C^-1 r.  Since T_p T_u = (T_{p+u} + T_{|p-u|}) / 2, G_pu = (S_{p+u} + S_{|p-u|}) / 2
// with S_k = sum_i mu_i^2 T_k(x_i) / C_i, k <= 2 order: each thread accumulates S and b in
// FP64 over its pixels (Chebyshev recurrence), the sums are reduced in a fixed order and
// stored, and a second kernel, one thread per row, solves M = G + Lambda^-1 by Cholesky in
// registers: the marginal form adds
// b^T M^-1 b / 2 - ln|M| / 2 - ln|Lambda| / 2 to logL, the optimised form c^T b - c^T G c / 2
// at c = M^-1 b (the diagonal likelihood at the regularised best fit).
// ---------------------------------------------------------------------------------
constexpr int kCalMax = 8;                 // coefficients at most (order 7)
constexpr int kCalS = 2 * kCalMax - 1;     // S_0 .. S_14

// The NC x NC solve of one row, unrolled so that everything stays in registers: G and b
// from the four waves' sums, Cholesky M = G + Lambda^-1 = L L^T, c = M^-1 b by two
// triangular solves, and the marginal or optimised correction.
template <int NC>
__device__ __forceinline__ double calib_solve(const double *__restrict__ sums, const DevObs &ob) {
  double G[NC][NC], M[NC][NC], b[NC], y[NC], c[NC];
  auto Sk = [&](int k) { return sums[k]; };
#pragma unroll
  for (int p = 0; p < NC; ++p) {
    b[p] = Sk(kCalS + p);
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      G[p][u] = 0.5 * (Sk(p + u) + Sk(p > u ? p - u : u - p));
      M[p][u] = G[p][u] + (p == u ? ob.calib_ivar[p] : 0.0);
    }
  }
  double logdet = 0.0;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    double s = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= M[j][k] * M[j][k];
    const double ljj = sqrt(s);
    M[j][j] = ljj;
    logdet += 2.0 * log(ljj);
#pragma unroll
    for (int i = j + 1; i < NC; ++i) {
      double t = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= M[i][k] * M[j][k];
      M[i][j] = t / ljj;
    }
  }
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    double t = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= M[i][k] * y[k];
    y[i] = t / M[i][i];
  }
#pragma unroll
  for (int i = NC - 1; i >= 0; --i) {
    double t = y[i];
#pragma unroll
    for (int k = i + 1; k < NC; ++k) t -= M[k][i] * c[k];
    c[i] = t / M[i][i];
  }
  double bc = 0.0, cGc = 0.0;
#pragma unroll
  for (int p = 0; p < NC; ++p) {
    bc += b[p] * c[p];
#pragma unroll
    for (int u = 0; u < NC; ++u) cGc += c[p] * G[p][u] * c[u];
  }
  return ob.calib_mode == 1 ? 0.5 * bc - 0.5 * logdet - ob.calib_lnsd : bc - 0.5 * cGc;
}

__global__ void __launch_bounds__(256) k_calib(DevLib lib, CalibLaunch a) {
  __shared__ double red[4][kCalS + kCalMax];
  const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const PointRow pr = a.rows[r];
  if (pr.b < 0) return;
  const DevObs &ob = a.obs_table[pr.obs];
  if (ob.kind != 1 || ob.calib_mode == 0) return;
  const int nc = ob.calib_order + 1;
  const double *th = a.theta + (size_t)pr.b * lib.P;
  const double ns = (ob.noise_flags & 1) ? exp(th[TH_LOG_ERR_SCALE]) : 1.0;
  const double fc = (ob.noise_flags & 2) ? exp(th[TH_LOG_F_CALIB]) : 0.0;
  const double fd = (ob.noise_flags & 4) ? exp(th[TH_LOG_F_DATA]) : 0.0;
  const double jt = (ob.noise_flags & 8) ? exp(th[TH_LOG_JITTER]) : 0.0;
  double S[kCalS], bv[kCalMax];
#pragma unroll
  for (int q = 0; q < kCalS; ++q) S[q] = 0.0;
#pragma unroll
  for (int q = 0; q < kCalMax; ++q) bv[q] = 0.0;
  const double *mu = a.msorted + (size_t)r * a.ld;
  for (int i = tid; i < ob.n_data; i += 256) {
    if (!ob.mask[i]) continue;
    const double m = mu[i], d = ob.data[i], sg = ob.sigma[i];
    const double v = ns * ns * sg * sg + fc * fc * m * m + fd * fd * d * d + jt * jt;
    const double w = 1.0 / v;
    const double q0 = m * m * w, r0 = m * (d - m) * w;
    const double x = ob.pix[i] * ob.calib_xs + ob.calib_x0;
    double t0 = 1.0, t1 = x;
    S[0] += q0;
    S[1] += q0 * x;
    bv[0] += r0;
    bv[1] += r0 * x;
#pragma unroll
    for (int k = 2; k < kCalS; ++k) {
      const double t2 = 2.0 * x * t1 - t0;
      S[k] += q0 * t2;
      if (k < kCalMax) bv[k] += r0 * t2;
      t0 = t1;
      t1 = t2;
    }
  }
  // fixed-order reduction: each wave by a butterfly, then the four waves in order
#pragma unroll
  for (int q = 0; q < kCalS; ++q) S[q] = wave_reduce_sum(S[q]);
#pragma unroll
  for (int q = 0; q < kCalMax; ++q) bv[q] = wave_reduce_sum(bv[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kCalS; ++q) red[wv][q] = S[q];
#pragma unroll
    for (int q = 0; q < kCalMax; ++q) red[wv][kCalS + q] = bv[q];
  }
  __syncthreads();
  for (int q = tid; q < kCalS + kCalMax; q += 256)
    a.sums[(size_t)r * a.ld_sums + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// One thread per sorted row: the row's solve (a kernel of its own, so that the unrolled
// solve's registers do not limit the occupancy of the sums)
__global__ void __launch_bounds__(64) k_calib_solve(CalibLaunch a) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= a.B_pad) return;
  const PointRow &pr = a.rows[r];
  if (pr.b < 0) return;
  const DevObs &ob = a.obs_table[pr.obs];
  if (ob.kind != 1 || ob.calib_mode == 0) return;
  const double *sums = a.sums + (size_t)r * a.ld_sums;
  double corr = 0.0;
  switch (ob.calib_order + 1) {
    case 1: corr = calib_solve<1>(sums, ob); break;
    case 2: corr = calib_solve<2>(sums, ob); break;
    case 3: corr = calib_solve<3>(sums, ob); break;
    case 4: corr = calib_solve<4>(sums, ob); break;
    case 5: corr = calib_solve<5>(sums, ob); break;
    case 6: corr = calib_solve<6>(sums, ob); break;
    case 7: corr = calib_solve<7>(sums, ob); break;
    default: corr = calib_solve<8>(sums, ob); break;
  }
  if (a.logl) a.logl[pr.b] += corr;
}

// ---------------------------------------------------------------------------------
// Analytic marginalisation of a spectrum's line fluxes (Sec. 4.1, App. I.3, eq.
// app_line_marg).  One workgroup per sorted row.  The fitted lines are those observed within
// the pixel range (a Gaussian-prior line with no grid flux stays fixed at 0), in wavelength
// order, at most kLineMargMax; line j's unit-flux profile on pixel i is
// A_ij = lambda_i / c N(ln lambda_i; ln lambda_j^obs, s_j) / f_nu^AB, taken within kLineCut
// s_j of the line as in the projection.  Phases:
//   1  per library line: grid flux, observed wavelength and width (spec_line_terms), the
//      fitted ones compacted in order by one wave (ballot prefix), each with its pixel window;
//   2  per pixel: W_i = 1 / sigma_eff^2 at the grid model (0 off the mask) and the residual
//      r_i = d_i - m_i plus the flat lines' grid profiles, into the row's scratch; the
//      diagonal likelihood of r;
//   3  b_j = sum_i A_ij W_i r_i (a wave per line) and P_jk = sum_i A_ij A_ik W_i over the
//      two windows' overlap (a wave per pair; pairs whose windows do not meet are 0), plus
//      s_j^-2 on the Gaussian lines' diagonal;
//   4  P = L L^T in LDS, right-looking, one column per step (a thread per row, rows outside
//      the band of overlapping lines skipped), with L y = b carried along:
//      ln Z = lnL_diag(r) + y^T y / 2 - sum ln L_jj - sum_G ln s_j + (m_flat / 2) ln 2 pi.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_linemarg(DevLib lib, LineMargLaunch a) {
  constexpr int NM = kLineMargMax;
  static_assert(NM <= 256, "the factorisation takes one row per thread");
  // the normal matrix's lower triangle, packed by rows (72 KB of LDS in all: two workgroups
  // per CU); before it is formed the same words hold the library lines' terms
  __shared__ double sPk[NM * (NM + 1) / 2];
  static_assert(NM * (NM + 1) / 2 >= 3 * 512 + 192, "the line terms fit where P goes");
  __shared__ double s_b[NM], s_F[NM], s_lnl[NM], s_isl[NM];
  __shared__ int s_p0[NM], s_p1[NM], s_aoff[NM], s_poff[NM + 1], s_atab;
  __shared__ unsigned char s_flat[NM];
  __shared__ short s_fidx[512];                  // library line -> fitted index, or -1
  __shared__ short s_lidx[NM];                   // fitted index -> library line
  __shared__ double s_pl;                        // joint with photometry: its lnL_diag
  __shared__ double s_cr[kLineCatMax], s_cw[kLineCatMax];   // joint: catalogue residuals, weights
  __shared__ double s_cl;                        // joint: the catalogue's -chi^2 / 2
  double *t_F = sPk, *t_lnl = sPk + 512, *t_sl = sPk + 1024;
  unsigned char *t_fit = (unsigned char *)(sPk + 1536), *t_flat = t_fit + 512, *t_cat = t_fit + 1024;
  auto P = [&](int i, int k) -> double & { return sPk[i * (i + 1) / 2 + k]; };   // k <= i
  __shared__ double red[4], s_lnsg;
  __shared__ int s_n, s_nflat;
  const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const PointRow &pr = a.rows[r];
  if (pr.b < 0) return;
  const DevObs &ob = a.obs_table[pr.obs];
  if (ob.kind != 1 || ob.lm_mode == 0) return;
  const double *th = a.theta + (size_t)pr.b * lib.P;
  const int nl = lib.n_line, np = ob.n_data;
  const double pix_lo = ob.pix[0], pix_hi = ob.pix[np - 1];
  // ---- 0. joint with a catalogue: the lines of its detected, included entries
  const DevObs *cat = a.cat;
  if (cat) {
    for (int l = tid; l < nl; l += 256) t_cat[l] = 0;
    __syncthreads();
    for (int e = tid; e < cat->n_data; e += 256)
      if (cat->mask[e] && !cat->upper[e])
        for (int q = cat->loff[e]; q < cat->loff[e + 1]; ++q) t_cat[cat->lidx[q]] = 1;
    __syncthreads();
  }
  // ---- 1. the library lines, then the fitted ones in order (the spectrum's, with a
  // catalogue also those of its detections)
  for (int l = tid; l < nl; l += 256) {
    double Fl, lobs, sl;
    spec_line_terms<true>(lib, ob, pr, th, a.Lline[(size_t)r * nl + l], l, Fl, lobs, sl);
    const bool flat = ob.lm_mode == 2 || (ob.lm_flat && ob.lm_flat[l]);
    t_F[l] = Fl;
    t_lnl[l] = log(lobs);
    t_sl[l] = sl;
    t_flat[l] = flat ? 1 : 0;
    const bool seen = (lobs >= pix_lo && lobs <= pix_hi) || (cat && t_cat[l]);
    t_fit[l] = (seen && (flat || Fl > 0.0)) ? 1 : 0;
    s_fidx[l] = -1;
  }
  __syncthreads();
  if (wv == 0) {
    int base = 0, nflat = 0;
    double lnsg = 0.0;
    for (int l0 = 0; l0 < nl; l0 += 64) {
      const int l = l0 + lane;
      const bool f = l < nl && t_fit[l];
      const unsigned long long m = __ballot(f);
      const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
      if (f && pos < NM) {
        s_fidx[l] = (short)pos;
        s_lidx[pos] = (short)l;
        s_F[pos] = t_F[l];
        s_lnl[pos] = t_lnl[l];
        s_isl[pos] = 1.0 / t_sl[l];
        s_flat[pos] = t_flat[l];
        const double w = kLineCut * t_sl[l];
        s_p0[pos] = lower_bound_dev(ob.lnpix, np, t_lnl[l] - w);
        int hi = lower_bound_dev(ob.lnpix, np, t_lnl[l] + w);
        while (hi < np && ob.lnpix[hi] <= t_lnl[l] + w) ++hi;
        s_p1[pos] = hi;
        if (t_flat[l]) ++nflat;
        else lnsg += log(ob.lm_frac * t_F[l]);
      }
      base += __popcll(m);
    }
    for (int o = 32; o > 0; o >>= 1) {
      nflat += __shfl_xor(nflat, o);
      lnsg += __shfl_xor(lnsg, o);
    }
    if (lane == 0) {
      s_n = min(base, NM);
      s_nflat = nflat;
      s_lnsg = lnsg;
    }
  }
  __syncthreads();
  const int n = s_n;
  // joint: each catalogue entry's residual at mu + A alpha_0 (the grid model, plus the grid
  // flux of its fitted flat lines) and weight; detections sum to the catalogue's -chi^2 / 2,
  // upper limits keep their one-sided form at the grid model (thread 0, entry order)
  if (cat && tid == 0) {
    double cl = 0.0;
    for (int e = 0; e < cat->n_data; ++e) {
      double rr = 0.0, w = 0.0;
      if (cat->mask[e]) {
        const double m = a.cat_model[(size_t)r * a.cat_ld + e], d = cat->data[e], sg = cat->sigma[e];
        if (cat->upper[e]) {
          if (m > d) cl -= 0.5 * ((d - m) / sg) * ((d - m) / sg);
        } else {
          rr = d - m;
          for (int q = cat->loff[e]; q < cat->loff[e + 1]; ++q) {
            const int j = s_fidx[cat->lidx[q]];
            if (j >= 0 && s_flat[j]) rr += s_F[j];
          }
          w = 1.0 / (sg * sg);
          cl -= 0.5 * rr * rr * w;
        }
      }
      s_cr[e] = rr;
      s_cw[e] = w;
    }
    s_cl = cl;
  }
  // joint with photometry: per band b and fitted line j the band response A_bj, the model
  // of line j alone per unit of its observed flux (its FP64 profile on the model grid
  // through the birth cloud with the escape factors, the diffuse screen, the IGM, the
  // observer frame and the filter nodes, as the projection forms the bands), in the row of
  // the photometric scratch; then each band's residual at mu + A alpha_0, weight and the
  // normalised Gaussian term of eq. 6 with the noise floor of eq. G1
  const DevObs *ph = a.phot;
  if (ph) {
    const int nb = ph->n_band, N = lib.N;
    double *pA = a.phot_scr + (size_t)r * a.phot_ld_scr, *pR = pA + (size_t)nb * NM, *pW = pR + nb;
    const double z = pr.z, opz = 1.0 + z, lnopz = log1p(z);
    const double fac = kC_cms * pr.scale_fnu / (opz * opz * kAng_cm * kAng_cm);
    const double Eb = 0.85 - 1.9 * pr.delta;
    const double wlo = lib.wave_d[0], whi = lib.wave_d[N - 1];
    for (int q = tid; q < nb * n; q += 256) {
      const int b = q / n, j = q - b * n, l = s_lidx[j];
      const int k0 = a.lprof_k0[l], kl = a.lprof_len[l];
      const double *prof = a.lprof + (size_t)l * a.lprof_w;
      const double Ll = a.Lline[(size_t)r * nl + l] / kLsun;
      auto Fline = [&](int k) {   // line l's rest-frame contribution at node k
        if (k < k0 || k >= k0 + kl) return 0.0;
        const double lv = lib.lnlv_d[k];
        const double td = exp(-pr.tau_diff * exp(pr.delta * lv) * (lib.dust_a_d[k] + Eb * lib.dust_d_d[k]));
        const double tb = pr.bc_p * exp(-pr.tau_bc * exp(pr.alpha_bc * lv)) + pr.bc_q;
        return td * tb * Ll * prof[k - k0] * igm_T(lib, th, z, lib.wave_d[k] * opz);
      };
      // the band's nodes whose bracketing interval touches the profile's nodes
      const double lo = lib.wave_d[max(k0 - 1, 0)] * opz, hi = lib.wave_d[min(k0 + kl, N - 1)] * opz;
      int n0 = ph->band_off[b], n1 = ph->band_off[b + 1];
      {
        int lo_i = n0, hi_i = n1;
        while (lo_i < hi_i) {
          const int mid = (lo_i + hi_i) >> 1;
          if (ph->fw[mid] < lo) lo_i = mid + 1; else hi_i = mid;
        }
        n0 = lo_i;
      }
      double sum = 0.0;
      for (int nn = n0; nn < n1 && ph->fw[nn] <= hi; ++nn) {
        const double lr = ph->fw[nn] / opz;
        if (!(lr >= wlo && lr <= whi)) continue;
        int k;
        if (lib.log_uniform) k = min(max((int)floor((ph->fwln[nn] - lnopz - lib.lnw0) * lib.inv_dlnw), 0), N - 2);
        else k = bracket(lib.wave_d, N, lr);
        const double w0 = lib.wave_d[k], w1 = lib.wave_d[k + 1];
        const double f0 = Fline(k), f1 = Fline(k + 1);
        const double t = (lr - w0) / (w1 - w0);
        sum += ph->fr_d[nn] * (f0 + t * (f1 - f0));
      }
      pA[(size_t)b * NM + j] = fac * sum / s_F[j];
    }
    __syncthreads();
    const double ns = (ph->noise_flags & 1) ? exp(th[TH_LOG_ERR_SCALE]) : 1.0;
    const double fcp = (ph->noise_flags & 2) ? exp(th[TH_LOG_F_CALIB]) : 0.0;
    const double fdp = (ph->noise_flags & 4) ? exp(th[TH_LOG_F_DATA]) : 0.0;
    const double jtp = (ph->noise_flags & 8) ? exp(th[TH_LOG_JITTER]) : 0.0;
    double lp = 0.0;
    for (int b = tid; b < nb; b += 256) {
      double rr = 0.0, w = 0.0;
      if (ph->mask[b]) {
        const double m = a.phot_model[(size_t)r * a.phot_ld + b], d = ph->data[b], sg = ph->sigma[b];
        const double v = ns * ns * sg * sg + fcp * fcp * m * m + fdp * fdp * d * d + jtp * jtp;
        w = 1.0 / v;
        rr = d - m;
        for (int j = 0; j < n; ++j)
          if (s_flat[j]) rr += s_F[j] * pA[(size_t)b * NM + j];
        lp += -0.5 * rr * rr * w - 0.5 * log(2.0 * kPi * v);
      }
      pR[b] = rr;
      pW[b] = w;
    }
    lp = wave_reduce_sum(lp);
    if (lane == 0) red[wv] = lp;
    __syncthreads();
    if (tid == 0) s_pl = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
  if (n == 0) {   // no line to fit: the grid model's likelihood stands (and the others')
    if (cat || ph) {
      __syncthreads();
      if (tid == 0 && a.logl) a.logl[pr.b] += (cat ? s_cl : 0.0) + (ph ? s_pl : 0.0);
    }
    return;
  }
  // unit-flux profile of fitted line j at pixel i (maggies per erg/s/cm^2)
  auto A = [&](int j, int i) {
    const double u = (ob.lnpix[i] - s_lnl[j]) * s_isl[j];
    return ob.pix[i] * (kAng_cm / kC_cms / kFnuAB) * (0.3989422804014327 * s_isl[j]) * exp(-0.5 * u * u);
  };
  // ---- 2. weights and residuals at the grid model; the diagonal likelihood of r
  const double ns = (ob.noise_flags & 1) ? exp(th[TH_LOG_ERR_SCALE]) : 1.0;
  const double fc = (ob.noise_flags & 2) ? exp(th[TH_LOG_F_CALIB]) : 0.0;
  const double fd = (ob.noise_flags & 4) ? exp(th[TH_LOG_F_DATA]) : 0.0;
  const double jt = (ob.noise_flags & 8) ? exp(th[TH_LOG_JITTER]) : 0.0;
  const double *mu = a.msorted + (size_t)r * a.ld;
  double *sr = a.scr + (size_t)r * a.ld_scr, *sw = sr + np;
  double lsum = 0.0;
  for (int i = tid; i < np; i += 256) {
    double w = 0.0, rr = 0.0;
    if (ob.mask[i]) {
      const double m = mu[i], d = ob.data[i], sg = ob.sigma[i];
      const double v = ns * ns * sg * sg + fc * fc * m * m + fd * fd * d * d + jt * jt;
      w = 1.0 / v;
      rr = d - m;
      if (s_nflat > 0)
        for (int j = 0; j < n; ++j)
          if (s_flat[j] && i >= s_p0[j] && i < s_p1[j]) rr += s_F[j] * A(j, i);
      lsum += -0.5 * rr * rr * w - 0.5 * log(2.0 * kPi * v);
    }
    sr[i] = rr;
    sw[i] = w;
  }
  lsum = wave_reduce_sum(lsum);
  if (lane == 0) red[wv] = lsum;
  __syncthreads();
  const double lnl_diag = (red[0] + red[1]) + (red[2] + red[3]);
  // ---- 3. b and the normal matrix P.  The profiles are tabulated once into the row's
  // scratch (after r and W) when they fit, line j's window at s_aoff[j].  The pairs (j, k),
  // k >= j, whose windows overlap (and every (j, j), which carries the prior) are counted per
  // line (thread j tests every k), numbered
  // by a scan and computed one per thread, each a serial sum over the overlap in pixel
  // order; the other entries are 0.
  double *abuf = sw + np;
  auto overlap = [&](int j, int k) { return k == j || (s_p0[k] < s_p1[j] && s_p0[j] < s_p1[k]); };
  for (int j = tid; j < n; j += 256) {
    int c = 0;
    for (int k = j; k < n; ++k) c += overlap(j, k) ? 1 : 0;
    s_aoff[j] = s_p1[j] - s_p0[j];   // window widths and pair counts, scanned below
    s_poff[j] = c;
  }
  for (int q = tid; q < n * (n + 1) / 2; q += 256) sPk[q] = 0.0;
  __syncthreads();
  if (wv == 0) {   // exclusive scans, 64 lines at a time
    int ca = 0, cp = 0;
    for (int j0 = 0; j0 < n; j0 += 64) {
      const int j = j0 + lane;
      int va = j < n ? s_aoff[j] : 0, vp = j < n ? s_poff[j] : 0;
      for (int o = 1; o < 64; o <<= 1) {
        const int ua = __shfl_up(va, o, 64), up = __shfl_up(vp, o, 64);
        if (lane >= o) {
          va += ua;
          vp += up;
        }
      }
      if (j < n) {
        s_aoff[j] = ca + va - s_aoff[j];
        s_poff[j] = cp + vp - s_poff[j];
      }
      ca += __shfl(va, 63, 64);
      cp += __shfl(vp, 63, 64);
    }
    if (lane == 0) {
      s_poff[n] = cp;
      s_atab = ca <= a.ld_scr - 2 * np ? 1 : 0;
    }
  }
  __syncthreads();
  const bool atab = s_atab != 0;
  if (atab) {
    const int total = s_aoff[n - 1] + (s_p1[n - 1] - s_p0[n - 1]);
    for (int t = tid; t < total; t += 256) {
      int lo = 0, hi = n - 1;   // the line whose window holds entry t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_aoff[mid] <= t) lo = mid; else hi = mid - 1;
      }
      abuf[t] = A(lo, s_p0[lo] + (t - s_aoff[lo]));
    }
    __syncthreads();
  }
  auto Ag = [&](int j, int i) { return atab ? abuf[s_aoff[j] + (i - s_p0[j])] : A(j, i); };
  // serial sums in pixel order, eight pixels' loads in flight at a time
  for (int j = tid; j < n; j += 256) {
    double acc = 0.0;
    int i = s_p0[j];
    const int up = s_p1[j];
    for (; i + 8 <= up; i += 8) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = Ag(j, i + u) * sw[i + u] * sr[i + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += x[u];
    }
    for (; i < up; ++i) acc += Ag(j, i) * sw[i] * sr[i];
    s_b[j] = acc;
  }
  const int npair = s_poff[n];
  for (int q = tid; q < npair; q += 256) {
    int j = 0, hi = n - 1;   // the pair's first line: the last j with s_poff[j] <= q
    while (j < hi) {
      const int mid = (j + hi + 1) >> 1;
      if (s_poff[mid] <= q) j = mid; else hi = mid - 1;
    }
    int k = j, m = q - s_poff[j];   // its m-th overlapping partner from j on
    while (true) {
      if (overlap(j, k)) {
        if (m == 0) break;
        --m;
      }
      ++k;
    }
    const int lo = max(s_p0[j], s_p0[k]), up = min(s_p1[j], s_p1[k]);
    double acc = 0.0;
    int i = lo;
    for (; i + 8 <= up; i += 8) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = Ag(j, i + u) * Ag(k, i + u) * sw[i + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += x[u];
    }
    for (; i < up; ++i) acc += Ag(j, i) * Ag(k, i) * sw[i];
    if (j == k && !s_flat[j]) {
      const double sj = ob.lm_frac * s_F[j];
      acc += 1.0 / (sj * sj);
    }
    P(k, j) = acc;
  }
  __syncthreads();
  if (cat && tid == 0) {   // the catalogue's detections: b_j += w r, P_jk += w for the fitted lines of a blend
    for (int e = 0; e < cat->n_data; ++e) {
      const double w = s_cw[e];
      if (w == 0.0) continue;
      for (int q = cat->loff[e]; q < cat->loff[e + 1]; ++q) {
        const int j = s_fidx[cat->lidx[q]];
        if (j < 0) continue;
        s_b[j] += w * s_cr[e];
        for (int q2 = cat->loff[e]; q2 < cat->loff[e + 1]; ++q2) {
          const int k = s_fidx[cat->lidx[q2]];
          if (k >= 0 && k <= j) P(j, k) += w;
        }
      }
    }
  }
  if (cat) __syncthreads();
  if (ph) {   // the photometry: b_j += sum_b w r A_bj, P_kj += sum_b w A_bj A_bk (bands in order)
    const int nb = ph->n_band;
    const double *pA = a.phot_scr + (size_t)r * a.phot_ld_scr, *pR = pA + (size_t)nb * NM, *pW = pR + nb;
    for (int j = tid; j < n; j += 256) {
      double acc = 0.0;
      for (int b = 0; b < nb; ++b) acc += pW[b] * pR[b] * pA[(size_t)b * NM + j];
      s_b[j] += acc;
    }
    for (int q = tid; q < n * (n + 1) / 2; q += 256) {   // q = k (k + 1) / 2 + j, j <= k
      int k = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while (k * (k + 1) / 2 > q) --k;
      while ((k + 1) * (k + 2) / 2 <= q) ++k;
      const int j = q - k * (k + 1) / 2;
      double acc = 0.0;
      for (int b = 0; b < nb; ++b) acc += pW[b] * pA[(size_t)b * NM + j] * pA[(size_t)b * NM + k];
      sPk[q] += acc;
    }
    __syncthreads();
  }
  // ---- 4. Cholesky with the forward solve carried along, one barrier per column: column j
  // (rows below the diagonal) and b_j are final when step j starts, and step j writes only
  // columns > j and b_i, i > j.  Every thread forms L_jj and y_j; thread i > j updates its row
  // of the lower triangle, P_ik -= L_ij L_kj for j < k <= i with L_kj = P_kj / L_jj, and b_i
  // (rows with L_ij = 0, outside the band of overlapping lines, skip)
  double sum_ln = 0.0, ssq = 0.0;   // thread 0
  for (int j = 0; j < n; ++j) {
    const double ljj = sqrt(P(j, j)), yj = s_b[j] / ljj, inv = 1.0 / ljj;
    if (tid == 0) {
      sum_ln += log(ljj);
      ssq += yj * yj;
    }
    const int i = j + 1 + tid;   // n <= 128 < 256: one row per thread
    if (i < n) {
      const double lij = P(i, j) * inv;
      if (lij != 0.0) {
        for (int k = j + 1; k <= i; ++k) P(i, k) -= lij * (P(k, j) * inv);
        s_b[i] -= lij * yj;
      }
    }
    __syncthreads();
  }
  if (tid == 0 && a.logl)
    a.logl[pr.b] = lnl_diag + (cat ? s_cl : 0.0) + (ph ? s_pl : 0.0) + 0.5 * ssq - sum_ln - s_lnsg +
                   0.5 * (double)s_nflat * log(2.0 * kPi);
}

hipError_t launch_linemarg(const DevLib &lib, const LineMargLaunch &lm, hipStream_t s) {
  if (lib.n_line > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_linemarg, dim3(lm.B_pad), dim3(256), 0, s, lib, lm);
  return hipGetLastError();
}

hipError_t launch_calib(const DevLib &lib, const CalibLaunch &cl, hipStream_t s) {
  if (cl.ld_sums < kCalS + kCalMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_calib, dim3(cl.B_pad), dim3(256), 0, s, lib, cl);
  hipLaunchKernelGGL(k_calib_solve, dim3((cl.B_pad + 63) / 64), dim3(64), 0, s, cl);
  return hipGetLastError();
}

hipError_t launch_project(const DevLib &lib, const ProjectLaunch &pl, hipStream_t s) {
  if (pl.f64) {
    ProjArgs<double> a{pl.obs_table, pl.rows, (const double *)pl.F, lib.N_pad, lib.n_line, pl.theta, pl.P, pl.B,
                       pl.Lline, pl.model, pl.logl, pl.gvec, pl.gnoise, pl.msorted, pl.ld_model, pl.ld_g};
    if (lib.igm) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project<double, true>), dim3(pl.B), dim3(256), 0, s, lib, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project<double, false>), dim3(pl.B), dim3(256), 0, s, lib, a);
  } else {
    ProjArgs<float> a{pl.obs_table, pl.rows, (const float *)pl.F, lib.N_pad, lib.n_line, pl.theta, pl.P, pl.B,
                      pl.Lline, pl.model, pl.logl, pl.gvec, pl.gnoise, pl.msorted, pl.ld_model, pl.ld_g};
    if (lib.igm) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project<float, true>), dim3(pl.B), dim3(256), 0, s, lib, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project<float, false>), dim3(pl.B), dim3(256), 0, s, lib, a);
  }
  return hipGetLastError();
}

}  // namespace sps
