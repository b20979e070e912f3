// Host runtime and C ABI of the batched SPS forward model (include/sps.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sps.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

namespace sps {

thread_local std::string g_last_error;

sps_status fail(sps_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

static int round_up(int x, int m) { return (x + m - 1) / m * m; }

DeviceArena::~DeviceArena() {
  if (base) (void)hipFree(base);
}
bool DeviceArena::init(size_t n) {
  n = (n + 255) / 256 * 256;
  if (hipMalloc((void **)&base, n) != hipSuccess) {
    base = nullptr;
    return false;
  }
  size = n;
  free_blocks.clear();
  free_blocks[0] = n;
  return true;
}
void *DeviceArena::alloc(size_t n) {
  n = (std::max<size_t>(n, 1) + 255) / 256 * 256;
  for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
    if (it->second < n) continue;
    const size_t off = it->first, len = it->second;
    free_blocks.erase(it);
    if (len > n) free_blocks[off + n] = len - n;
    return base + off;
  }
  return nullptr;
}
void DeviceArena::free(void *p, size_t n) {
  n = (std::max<size_t>(n, 1) + 255) / 256 * 256;
  size_t off = (size_t)((char *)p - base);
  auto nx = free_blocks.lower_bound(off);
  if (nx != free_blocks.end() && off + n == nx->first) {   // merge with the block after
    n += nx->second;
    nx = free_blocks.erase(nx);
  }
  if (nx != free_blocks.begin()) {   // and with the block before
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      off = pv->first;
      n += pv->second;
      free_blocks.erase(pv);
    }
  }
  free_blocks[off] = n;
}

DeviceBuffers::~DeviceBuffers() { release(); }
void DeviceBuffers::release() {
  for (size_t k = 0; k < ptrs.size(); ++k) {
    if (arena) arena->free(ptrs[k], sizes[k]);
    else (void)hipFree(ptrs[k]);
  }
  ptrs.clear();
  sizes.clear();
  bytes = 0;
}
void *DeviceBuffers::alloc(size_t n) {
  if (n == 0) n = 16;
  void *p = nullptr;
  if (arena) {
    p = arena->alloc(n);
    if (!p) return nullptr;
  } else if (hipMalloc(&p, n) != hipSuccess) {
    return nullptr;
  }
  ptrs.push_back(p);
  sizes.push_back(n);
  bytes += (int64_t)n;
  return p;
}
void *DeviceBuffers::upload(const void *h, size_t n) {
  void *p = alloc(n);
  if (p && h && hipMemcpy(p, h, n, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return p;
}

// Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n (n = 16).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

static bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}
static bool increasing(const double *p, size_t n) {
  for (size_t i = 1; i < n; ++i)
    if (!(p[i] > p[i - 1])) return false;
  return true;
}

}  // namespace sps

using namespace sps;

// =====================================================================================
// Library
// =====================================================================================
extern "C" sps_status sps_library_load(const sps_library_desc *d, sps_library **out) {
  if (!d || !out) return fail(SPS_E_INVAL, "sps_library_load: NULL argument");
  *out = nullptr;
  const int na = d->n_age, nz = d->n_z, nf = d->n_afe, N = d->n_wave;
  if (na < 2 || nz < 1 || nf < 1 || N < 2) return fail(SPS_E_SHAPE, "library needs n_age>=2, n_z>=1, n_afe>=1, n_wave>=2");
  if (!d->ages || !d->logz || !d->wave || !d->flux) return fail(SPS_E_INVAL, "library arrays must not be NULL");
  if (nf > 1 && !d->afe) return fail(SPS_E_INVAL, "afe nodes required when n_afe > 1");
  if (!finite_all(d->ages, na) || !increasing(d->ages, na) || d->ages[0] <= 0)
    return fail(SPS_E_INVAL, "ages must be finite, positive and strictly increasing");
  if (!finite_all(d->logz, nz) || !increasing(d->logz, nz)) return fail(SPS_E_INVAL, "logz must be strictly increasing");
  if (nf > 1 && (!finite_all(d->afe, nf) || !increasing(d->afe, nf)))
    return fail(SPS_E_INVAL, "afe must be strictly increasing");
  if (!finite_all(d->wave, N) || !increasing(d->wave, N) || d->wave[0] <= 0)
    return fail(SPS_E_INVAL, "wave must be positive and strictly increasing");
  const size_t nflux = (size_t)nf * nz * na * N;
  for (size_t i = 0; i < nflux; ++i)
    if (!std::isfinite(d->flux[i]) || d->flux[i] < 0) return fail(SPS_E_INVAL, "flux must be finite and >= 0");
  if (d->n_sfh < 2 || d->n_sfh > 1024) return fail(SPS_E_SHAPE, "n_sfh must be in [2, 1024]");
  if (d->n_zh < 0 || d->n_zh == 1 || d->n_zh > 1024) return fail(SPS_E_SHAPE, "n_zh must be 0 or in [2, 1024]");
  if (!(d->T1 > 0) || !(d->H0 > 0) || !(d->Om > 0 && d->Om < 1) || !(d->t_young > 0))
    return fail(SPS_E_INVAL, "T1, H0, t_young must be > 0 and 0 < Om < 1");
  int ny = 0;
  while (ny < na && d->ages[ny] < d->t_young) ++ny;
  const int nl = d->n_line;
  if (nl < 0 || nl > 512) return fail(SPS_E_SHAPE, "n_line must be in [0, 512]");
  if (nl > 0) {
    if (!d->line_wave || !d->line_table || !d->zg_nodes || !d->u_nodes || d->n_zg < 2 || d->n_u < 2)
      return fail(SPS_E_INVAL, "line tables incomplete");
    if (ny == 0) return fail(SPS_E_INVAL, "nebular lines need SSP ages younger than t_young");
    if (!increasing(d->line_wave, nl) || !increasing(d->zg_nodes, d->n_zg) || !increasing(d->u_nodes, d->n_u))
      return fail(SPS_E_INVAL, "line wavelengths and table axes must be strictly increasing");
    if (d->n_line_tau < 0 || (d->n_line_tau > 0 && (d->n_line_tau < 2 || !d->line_tau)))
      return fail(SPS_E_INVAL, "line_tau needs n_line_tau >= 2 ages");
    if (d->n_line_tau > 0 && (!finite_all(d->line_tau, d->n_line_tau) || !increasing(d->line_tau, d->n_line_tau)))
      return fail(SPS_E_INVAL, "line_tau must be finite and strictly increasing");
    const int nlt = d->n_line_tau > 0 ? d->n_line_tau : ny;
    if (!finite_all(d->line_table, (size_t)nl * nlt * d->n_zg * d->n_u)) return fail(SPS_E_INVAL, "line table not finite");
  }
  const bool has_cont = d->n_cont_tau > 0;
  if (has_cont) {
    if (d->n_cont_tau < 2 || d->n_cont_zg < 2 || d->n_cont_u < 2 || !d->cont_tau || !d->cont_zg || !d->cont_u ||
        !d->cont_table)
      return fail(SPS_E_INVAL, "nebular continuum cube incomplete (each axis needs >= 2 nodes)");
    if (!finite_all(d->cont_tau, d->n_cont_tau) || !increasing(d->cont_tau, d->n_cont_tau) ||
        !finite_all(d->cont_zg, d->n_cont_zg) || !increasing(d->cont_zg, d->n_cont_zg) ||
        !finite_all(d->cont_u, d->n_cont_u) || !increasing(d->cont_u, d->n_cont_u))
      return fail(SPS_E_INVAL, "nebular continuum axes must be finite and strictly increasing");
    if ((int64_t)d->n_cont_zg * d->n_cont_u > 128) return fail(SPS_E_SHAPE, "nebular continuum cube: at most 128 (Z_gas, U) nodes");
    if (!finite_all(d->cont_table, (size_t)d->n_cont_tau * d->n_cont_zg * d->n_cont_u * N))
      return fail(SPS_E_INVAL, "nebular continuum cube not finite");
  }
  if (d->escape < SPS_ESCAPE_NONE || d->escape > SPS_ESCAPE_PICKET) return fail(SPS_E_INVAL, "unknown escape geometry");
  if (d->sfh_scheme != SPS_SFH_STEP && d->sfh_scheme != SPS_SFH_LINEAR) return fail(SPS_E_INVAL, "unknown SFH scheme");
  if (d->igm != 0 && d->igm != 1 && d->igm != 3 && d->igm != 5 && d->igm != 7)
    return fail(SPS_E_INVAL, "igm: 0, or SPS_IGM_MADAU with optional SPS_IGM_DAMPING and SPS_IGM_DLA");
  if (!(d->sigma_gal_max >= 0) || !std::isfinite(d->sigma_gal_max))
    return fail(SPS_E_INVAL, "sigma_gal_max must be finite and >= 0");
  if (d->sigma_gal_max > 0) {
    // the Fourier stage's uniform ln(lambda) grid is the model grid itself
    const double dl = (std::log(d->wave[N - 1]) - std::log(d->wave[0])) / (N - 1);
    for (int n = 0; n + 1 < N; ++n)
      if (std::fabs((std::log(d->wave[n + 1]) - std::log(d->wave[n])) / dl - 1.0) >= 1e-6)
        return fail(SPS_E_INVAL, "a free sigma_gal needs a wavelength grid uniform in ln(lambda)");
  }
  // nebular-covered SSP ages [neb_a0, neb_a1): inside every cube's age range (App. C)
  int neb_a0 = 0, neb_a1 = 0;
  if (nl > 0 || has_cont) {
    double lo = -HUGE_VAL, hi = HUGE_VAL;
    if (nl > 0) {
      lo = std::max(lo, d->n_line_tau > 0 ? d->line_tau[0] : d->ages[0]);
      hi = std::min(hi, d->n_line_tau > 0 ? d->line_tau[d->n_line_tau - 1] : d->ages[ny - 1]);
    }
    if (has_cont) {
      lo = std::max(lo, d->cont_tau[0]);
      hi = std::min(hi, d->cont_tau[d->n_cont_tau - 1]);
    }
    while (neb_a0 < na && d->ages[neb_a0] < lo) ++neb_a0;
    neb_a1 = neb_a0;
    while (neb_a1 < na && d->ages[neb_a1] <= hi) ++neb_a1;
    if (neb_a1 <= neb_a0) return fail(SPS_E_INVAL, "no SSP age falls inside the nebular grids' age range");
    if (neb_a1 > ny) return fail(SPS_E_INVAL, "nebular-covered SSP ages must be birth-cloud ages (younger than t_young)");
    if (has_cont && neb_a1 - neb_a0 > 128) return fail(SPS_E_SHAPE, "at most 128 nebular-covered SSP ages with a continuum");
  }
  if (d->device >= 0) {
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || d->device >= dev_count)
      return fail(SPS_E_HIP, "no HIP device %d", d->device);
    if (hipSetDevice(d->device) != hipSuccess) return fail(SPS_E_HIP, "hipSetDevice(%d) failed", d->device);
  }

  auto *L = new sps_library();
  L->device = d->device;
  L->n_age = na;
  L->n_z = nz;
  L->n_afe = nf;
  L->N = N;
  L->n_young = ny;
  L->n_line = nl;
  L->n_sfh = d->n_sfh;
  L->n_zh = d->n_zh;
  L->line_tau_axis = nl > 0 && d->n_line_tau > 0;
  L->precisions = d->precisions | (1u << SPS_FP32);
  L->wave_h.assign(d->wave, d->wave + N);
  if (nl > 0) L->line_wave_h.assign(d->line_wave, d->line_wave + nl);
  L->logz_lo = d->logz[0];
  L->logz_hi = d->logz[nz - 1];
  L->afe_lo = nf > 1 ? d->afe[0] : 0.0;
  L->afe_hi = nf > 1 ? d->afe[nf - 1] : 0.0;
  DevLib &g = L->dev;
  memset(&g, 0, sizeof g);
  g.n_age = na;
  g.n_z = nz;
  g.n_afe = nf;
  g.N = N;
  g.N_pad = round_up(N, kNAlign);
  g.n_young = ny;
  g.n_line = nl;
  g.n_zg = nl ? d->n_zg : 0;
  g.n_u = nl ? d->n_u : 0;
  g.n_sfh = d->n_sfh;
  g.n_zh = d->n_zh;
  const int igm_cols = (d->igm & 1) + ((d->igm >> 1) & 1) + 2 * ((d->igm >> 2) & 1);
  g.P = TH_NSCALAR + d->n_sfh + d->n_zh + (d->escape ? 1 : 0) + igm_cols + (d->sigma_gal_max > 0 ? 1 : 0);
  g.th_fob = TH_NSCALAR + d->n_sfh + d->n_zh;
  g.th_igm = g.th_fob + (d->escape ? 1 : 0);
  g.igm = d->igm;
  g.th_xhi = g.th_igm + 1;
  g.th_nhi = g.th_xhi + ((d->igm >> 1) & 1);
  g.vdisp = d->sigma_gal_max > 0 ? 1 : 0;
  g.th_sgal = g.th_igm + igm_cols;
  g.vd_max = d->sigma_gal_max;
  g.sfh_scheme = d->sfh_scheme;
  g.escape = d->escape;
  g.neb_a0 = neb_a0;
  g.neb_a1 = neb_a1;
  g.has_neb = (nl > 0 || has_cont) ? 1 : 0;
  g.has_cont = has_cont ? 1 : 0;
  g.n_cz = has_cont ? d->n_cont_zg : 0;
  g.n_cu = has_cont ? d->n_cont_u : 0;
  g.ion_nlim = N;
  for (int n = 0; n < N; ++n)
    if (d->wave[n] >= kLamLyman) {
      g.ion_nlim = n;
      break;
    }
  g.T1 = d->T1;
  g.H0 = d->H0;
  g.Om = d->Om;
  g.t_young = d->t_young;

  // ---- young-first K order.  Time-varying enrichment: age-major (old ages beyond
  //      t_univ(z) form whole zero tiles); constant metallicity: metallicity-major
  //      (rows of one metallicity/alpha bracket share a few (Z, alpha) blocks).
  //      With an escape geometry the raw ionising continuum of the nebular ages follows
  //      the young segment as rows of its own (ion rows, age-major); under the picket
  //      fence the line rows start on a K tile of their own, so that the dust-free pass
  //      can take the young stellar rows without them.
  const int kyo = ny * nz * nf;
  const int line_k0 = d->escape == SPS_ESCAPE_PICKET ? round_up(kyo, kKAlign) : kyo;
  const int K_young_pad = round_up(line_k0 + nl, kKAlign);
  const int n_ion = d->escape ? (neb_a1 - neb_a0) * nz * nf : 0;
  const int K_old0 = K_young_pad + round_up(n_ion, kKAlign);
  const int kold = (na - ny) * nz * nf;
  const int K_pad = K_old0 + round_up(kold, kKAlign);
  g.K = nf * nz * na + nl;
  g.K_pad = K_pad;
  if (K_pad > kMaxKPad) return fail(SPS_E_SHAPE, "library too large: %d weight rows after padding (at most %d)", K_pad, kMaxKPad);
  g.K_young_pad = K_young_pad;
  g.line_k0 = line_k0;
  g.ion_k0 = K_young_pad;
  g.n_ion = n_ion;
  g.K_old0 = K_old0;
  std::vector<int> kpos((size_t)nf * nz * na), ksrc(K_pad, INT_MIN);
  g.zmajor = d->n_zh > 0 ? 0 : 1;
  auto place = [&](int a0, int a1, int kbase) {
    int k = kbase;
    if (d->n_zh > 0) {
      for (int a = a0; a < a1; ++a)
        for (int m = 0; m < nz; ++m)
          for (int ia = 0; ia < nf; ++ia) kpos[(ia * nz + m) * na + a] = k++;
    } else {
      for (int m = 0; m < nz; ++m)
        for (int ia = 0; ia < nf; ++ia)
          for (int a = a0; a < a1; ++a) kpos[(ia * nz + m) * na + a] = k++;
    }
  };
  place(0, ny, 0);
  place(ny, na, K_old0);
  for (int s = 0; s < nf * nz * na; ++s) ksrc[kpos[s]] = s;
  L->line_k0 = line_k0;
  for (int l = 0; l < nl; ++l) ksrc[line_k0 + l] = -1 - l;
  for (int q = 0; q < n_ion; ++q) {   // ion row q: ((a - neb_a0) * nz + m) * nf + ia
    const int ia = q % nf, m = (q / nf) % nz, a = neb_a0 + q / (nf * nz);
    ksrc[K_young_pad + q] = kIonSrc - ((ia * nz + m) * na + a);
  }

  if (d->device < 0) {   // host-only library: layout and observation operators only
    L->precisions = 0;
    *out = L;
    return SPS_OK;
  }

  // ---- static per-wavelength tables
  const int Np = g.N_pad;
  std::vector<double> wave(Np), lnw(Np), lnlv(Np, 0.0), da(Np, 0.0), dd(Np, 0.0), lam2(Np, 0.0);
  std::vector<float> wave_f(Np), lnlv_f(Np, 0.f), da_f(Np, 0.f), dd_f(Np, 0.f);
  for (int n = 0; n < Np; ++n) {
    const bool in = n < N;
    wave[n] = in ? d->wave[n] : d->wave[N - 1] * (1.0 + 1e-3 * (n - N + 1));
    lnw[n] = std::log(wave[n]);
    if (in) {
      lnlv[n] = std::log(d->wave[n] / kLamV);
      da[n] = d->dust_a ? d->dust_a[n] : 0.0;
      dd[n] = d->dust_d ? d->dust_d[n] : 0.0;
      lam2[n] = d->wave[n] * d->wave[n];
    }
    wave_f[n] = (float)wave[n];
    lnlv_f[n] = (float)lnlv[n];
    da_f[n] = (float)da[n];
    dd_f[n] = (float)dd[n];
  }
  {
    const double dl = (std::log(d->wave[N - 1]) - std::log(d->wave[0])) / (N - 1);
    double dev = 0.0;
    for (int n = 0; n + 1 < N; ++n)
      dev = std::max(dev, std::fabs((std::log(d->wave[n + 1]) - std::log(d->wave[n])) / dl - 1.0));
    g.log_uniform = dev < 1e-6 ? 1 : 0;
    g.lnw0 = std::log(d->wave[0]);
    g.inv_dlnw = 1.0 / dl;
    g.dlnw = dl;
  }
  // Voronoi cells of the age nodes (App. B): first from 0, last to +inf
  std::vector<double> lo(na), hi(na);
  for (int a = 0; a < na; ++a) {
    lo[a] = a == 0 ? 0.0 : 0.5 * (d->ages[a - 1] + d->ages[a]);
    hi[a] = a == na - 1 ? HUGE_VAL : 0.5 * (d->ages[a] + d->ages[a + 1]);
  }
  // composite Gauss-Legendre on [0, 1]: 8 panels x 16 nodes
  std::vector<double> gx, gw, glu, glw;
  gauss_legendre(16, gx, gw);
  const int panels = 8;
  for (int p = 0; p < panels; ++p)
    for (int i = 0; i < 16; ++i) {
      glu.push_back((p + 0.5 * (gx[i] + 1.0)) / panels);
      glw.push_back(0.5 * gw[i] / panels);
    }
  g.n_gl = (int)glu.size();
  // line profiles on the model grid: Gaussian of sigma = 2 local pixels, truncated at
  // 5 sigma, unit trapezoid integral (Sec. 2.3.1, App. C)
  std::vector<double> lineprof, line_a(std::max(nl, 1)), line_d(std::max(nl, 1));
  if (nl > 0) {
    lineprof.assign((size_t)nl * N, 0.0);
    std::vector<double> tw(N, 0.0);
    for (int n = 0; n + 1 < N; ++n) {
      const double h = 0.5 * (d->wave[n + 1] - d->wave[n]);
      tw[n] += h;
      tw[n + 1] += h;
    }
    for (int l = 0; l < nl; ++l) {
      const double lw = d->line_wave[l];
      int k = (int)(std::upper_bound(d->wave, d->wave + N, lw) - d->wave) - 1;
      k = std::min(std::max(k, 0), N - 2);
      const double sg = 2.0 * (d->wave[k + 1] - d->wave[k]);
      double norm = 0.0;
      double *row = lineprof.data() + (size_t)l * N;
      for (int n = 0; n < N; ++n) {
        const double x = d->wave[n] - lw;
        if (std::fabs(x) <= 5.0 * sg) {
          row[n] = std::exp(-0.5 * (x / sg) * (x / sg));
          norm += row[n] * tw[n];
        }
      }
      for (int n = 0; n < N; ++n) row[n] /= norm;
      // dust shape tables at the line wavelength (linear in lambda, clamped)
      auto interp = [&](const double *tab) {
        if (!tab) return 0.0;
        if (lw <= d->wave[0]) return tab[0];
        if (lw >= d->wave[N - 1]) return tab[N - 1];
        const int j = (int)(std::upper_bound(d->wave, d->wave + N, lw) - d->wave) - 1;
        const double t = (lw - d->wave[j]) / (d->wave[j + 1] - d->wave[j]);
        return tab[j] + t * (tab[j + 1] - tab[j]);
      };
      line_a[l] = interp(d->dust_a);
      line_d[l] = interp(d->dust_d);
    }
  }

  const size_t prep_lds = std::max(prep_smem_bytes(g, 0), prep_smem_bytes(g, 3));
  if (prep_lds > 160 * 1024)
    return fail(SPS_E_SHAPE, "library too large for the per-point weight builder (%zu bytes of LDS)", prep_lds);
  // ---- device copies
  DeviceBuffers &mem = L->mem;
  bool ok = true;
  auto up = [&](const void *h, size_t n) {
    void *p = mem.upload(h, n);
    ok = ok && p;
    return p;
  };
  auto al = [&](size_t n) {
    void *p = mem.alloc(n);
    ok = ok && p;
    return p;
  };
  g.cell_lo = (const double *)up(lo.data(), na * 8);
  g.cell_hi = (const double *)up(hi.data(), na * 8);
  g.logz = (const double *)up(d->logz, nz * 8);
  std::vector<double> afe(nf, 0.0);
  if (nf > 1) std::copy(d->afe, d->afe + nf, afe.begin());
  g.afe = (const double *)up(afe.data(), nf * 8);
  g.wave_d = (const double *)up(wave.data(), Np * 8);
  g.lnwave_d = (const double *)up(lnw.data(), Np * 8);
  g.wave_f = (const float *)up(wave_f.data(), Np * 4);
  g.lnlv_d = (const double *)up(lnlv.data(), Np * 8);
  g.lnlv_f = (const float *)up(lnlv_f.data(), Np * 4);
  g.dust_a_d = (const double *)up(da.data(), Np * 8);
  g.dust_d_d = (const double *)up(dd.data(), Np * 8);
  g.dust_a_f = (const float *)up(da_f.data(), Np * 4);
  g.dust_d_f = (const float *)up(dd_f.data(), Np * 4);
  g.lam2_d = (const double *)up(lam2.data(), Np * 8);
  g.gl_u = (const double *)up(glu.data(), glu.size() * 8);
  g.gl_w = (const double *)up(glw.data(), glw.size() * 8);
  if (nl > 0) {   // the line profiles' nonzero nodes, compactly (joint marginalisation with photometry)
    std::vector<int> k0(nl, 0), len(nl, 0);
    int wmax = 1;
    for (int l = 0; l < nl; ++l) {
      const double *row = lineprof.data() + (size_t)l * N;
      int a = 0, b = N - 1;
      while (a < N && row[a] == 0.0) ++a;
      while (b > a && row[b] == 0.0) --b;
      k0[l] = a < N ? a : 0;
      len[l] = a < N ? b - a + 1 : 0;
      wmax = std::max(wmax, len[l]);
    }
    std::vector<double> prof((size_t)nl * wmax, 0.0);
    for (int l = 0; l < nl; ++l)
      for (int q = 0; q < len[l]; ++q) prof[(size_t)l * wmax + q] = lineprof[(size_t)l * N + k0[l] + q];
    L->lprof_w = wmax;
    L->lprof_d = (const double *)up(prof.data(), prof.size() * 8);
    L->lprof_k0_d = (const int *)up(k0.data(), nl * 4);
    L->lprof_len_d = (const int *)up(len.data(), nl * 4);
  }
  L->kpos_d = (int *)up(kpos.data(), kpos.size() * 4);
  int *ksrc_d = (int *)up(ksrc.data(), ksrc.size() * 4);
  // the weight builder's node tables in one block, in its LDS order (DevLib::prep_tab);
  // with lines on, the photon rates Q close the block and are written by the packing
  std::vector<double> ptab((size_t)prep_tab_len(g), 0.0);
  {
    size_t o = 0;
    for (int m = 0; m < nz; ++m) ptab[o++] = d->logz[m];
    for (int m = 0; m < nf; ++m) ptab[o++] = afe[m];
    for (int a = 0; a < na; ++a) ptab[o++] = lo[a];
    for (int a = 0; a < na; ++a) ptab[o++] = hi[a];
    for (int m = 0; m < g.n_zg; ++m) ptab[o++] = d->zg_nodes[m];
    for (int m = 0; m < g.n_u; ++m) ptab[o++] = d->u_nodes[m];
    if (g.sfh_scheme) {   // the ages close the block, after Q (written by the packing)
      size_t oa = o + (g.has_neb ? (size_t)nf * nz * ny : 0);
      for (int a = 0; a < na; ++a) ptab[oa++] = d->ages[a];
    }
  }
  double *ptab_d = (double *)up(ptab.data(), ptab.size() * 8);
  g.prep_tab = ptab_d;
  const size_t q_off = (size_t)nz + nf + 2 * na + g.n_zg + g.n_u;
  double *Q = g.has_neb ? (ptab_d ? ptab_d + q_off : nullptr) : (double *)al((size_t)std::max(1, nf * nz * ny) * 8);
  g.Q = Q;
  // bracketing node j and fraction t of x on an increasing axis, clamped (the age step of
  // the cubes' trilinear interpolation, done once here for the fixed SSP ages)
  auto split = [](const double *x, int n, double v, int &j, double &t) {
    const double vc = std::min(std::max(v, x[0]), x[n - 1]);
    j = 0;
    while (j + 1 < n - 1 && x[j + 1] <= vc) ++j;
    t = (vc - x[j]) / (x[j + 1] - x[j]);
  };
  if (nl > 0) {
    // stored as [zg][u][line][young age]: for one (Z_gas, U) corner the (line, age) slab is
    // contiguous.  A table with an age axis of its own is interpolated linearly in age at
    // each nebular SSP age; young ages outside the nebular range take -1000 (10^-1000 = 0).
    const int nlt = d->n_line_tau > 0 ? d->n_line_tau : ny;
    std::vector<double> ltT((size_t)nl * ny * d->n_zg * d->n_u);
    for (int a = 0; a < ny; ++a) {
      int j = a;
      double t = 0.0;
      if (d->n_line_tau > 0 && a >= neb_a0 && a < neb_a1) split(d->line_tau, nlt, d->ages[a], j, t);
      for (int l = 0; l < nl; ++l)
        for (int ig = 0; ig < d->n_zg; ++ig)
          for (int iu = 0; iu < d->n_u; ++iu) {
            double v = -1000.0;
            if (a >= neb_a0 && a < neb_a1) {
              auto at = [&](int jt) { return d->line_table[(((size_t)l * nlt + jt) * d->n_zg + ig) * d->n_u + iu]; };
              v = d->n_line_tau > 0 ? (1.0 - t) * at(j) + t * at(j + 1) : at(a);
            }
            ltT[(((size_t)ig * d->n_u + iu) * nl + l) * ny + a] = v;
          }
    }
    g.line_table = (const double *)up(ltT.data(), ltT.size() * 8);
    std::vector<float> ltF(ltT.begin(), ltT.end());
    g.line_table_f = (const float *)up(ltF.data(), ltF.size() * 4);
    g.zg = (const double *)up(d->zg_nodes, d->n_zg * 8);
    g.un = (const double *)up(d->u_nodes, d->n_u * 8);
    g.line_wave = (const double *)up(d->line_wave, nl * 8);
    g.line_a = (const double *)up(line_a.data(), nl * 8);
    g.line_d = (const double *)up(line_d.data(), nl * 8);
  }
  if (has_cont) {
    // nebular continuum: the cube interpolated linearly in age at each nebular SSP age,
    // [age][zg][u][N_pad]; per pixel the largest value c_ref is taken out (FP32: every
    // term 2^x has x <= 0) and 10^{c_ref} c / lambda^2 / Lsun * kWqScale kept apart
    const int nct = d->n_cont_tau, ncz = d->n_cont_zg, ncu = d->n_cont_u, n_nc = neb_a1 - neb_a0;
    const size_t plane = (size_t)ncz * ncu;
    std::vector<double> cres((size_t)n_nc * plane * Np, 0.0), cref(Np, -HUGE_VAL);
    for (int q = 0; q < n_nc; ++q) {
      int j;
      double t;
      split(d->cont_tau, nct, d->ages[neb_a0 + q], j, t);
      for (size_t c = 0; c < plane; ++c)
        for (int n = 0; n < N; ++n) {
          const double v = (1.0 - t) * d->cont_table[((size_t)j * plane + c) * N + n] +
                           t * d->cont_table[((size_t)(j + 1) * plane + c) * N + n];
          cres[((size_t)q * plane + c) * Np + n] = v;
          cref[n] = std::max(cref[n], v);
        }
    }
    std::vector<double> cd(cres.size()), scd(Np, 0.0);
    std::vector<float> cf(cres.size()), scf(Np, 0.f);
    const double log2_10 = 3.321928094887362347870319429489390175864831393;
    for (size_t i = 0; i < cres.size(); ++i) {
      const int n = (int)(i % Np);
      const double x = n < N ? cres[i] - cref[n] : -1000.0;
      cd[i] = x;
      cf[i] = (float)(x * log2_10);
    }
    for (int n = 0; n < N; ++n) {
      scd[n] = std::pow(10.0, cref[n]) * (kC_cms / kAng_cm) / (d->wave[n] * d->wave[n]) / kLsun * kWqScale;
      scf[n] = (float)scd[n];
    }
    g.cz = (const double *)up(d->cont_zg, ncz * 8);
    g.cu = (const double *)up(d->cont_u, ncu * 8);
    if (L->precisions & (1u << SPS_FP64)) {
      g.cont_d = (const double *)up(cd.data(), cd.size() * 8);
      g.cont_sc_d = (const double *)up(scd.data(), Np * 8);
    }
    g.cont_f = (const float *)up(cf.data(), cf.size() * 4);
    g.cont_sc_f = (const float *)up(scf.data(), Np * 4);
  }
  int *kexp = (int *)al((size_t)K_pad * 4);
  g.kexp = kexp;
  int16_t *kexp16 = (int16_t *)al((size_t)K_pad * 2);
  g.kexp16 = kexp16;
  const size_t KN = (size_t)K_pad * Np;
  PackLaunch pk;
  memset(&pk, 0, sizeof pk);
  pk.LT32 = (float *)al(KN * 4);
  pk.L32n = (float *)al(KN * 4);
  if (L->precisions & (1u << SPS_FP64)) pk.LT64 = (double *)al(KN * 8);
  const uint32_t bf_set = (1u << SPS_BF16) | (1u << SPS_BF16_1PASS) | (1u << SPS_BF16_HR) | (1u << SPS_BF16_WL);
  const uint32_t h_set = (1u << SPS_FP16) | (1u << SPS_FP16_1PASS) | (1u << SPS_FP16_HR) | (1u << SPS_FP16_WL);
  const bool want_bf = L->precisions & bf_set;
  const bool want_h = L->precisions & h_set;
  if (want_bf) {
    pk.Hb = (uint16_t *)al(KN * 2);
    pk.Rb = (uint16_t *)al(KN * 2);
    L->precisions |= bf_set;
  }
  if (want_h) {
    pk.Hh = (uint16_t *)al(KN * 2);
    pk.Rh = (uint16_t *)al(KN * 2);
    L->precisions |= h_set;
  }
  if (!ok) {
    delete L;
    return fail(SPS_E_NOMEM, "sps_library_load: device allocation failed");
  }
  g.LT64 = pk.LT64;
  g.LT32 = pk.LT32;
  g.L32n = pk.L32n;
  g.Hb = pk.Hb;
  g.Rb = pk.Rb;
  g.Hh = pk.Hh;
  g.Rh = pk.Rh;
  // temporary uploads of the raw grid and the line profiles
  DeviceBuffers tmp;
  pk.flux = (const double *)tmp.upload(d->flux, nflux * 8);
  pk.lineprof = nl ? (const double *)tmp.upload(lineprof.data(), lineprof.size() * 8) : nullptr;
  if (!pk.flux || (nl && !pk.lineprof)) {
    delete L;
    return fail(SPS_E_NOMEM, "sps_library_load: staging allocation failed");
  }
  pk.ksrc = ksrc_d;
  pk.neb_mask = g.has_neb;
  pk.kexp = kexp;
  pk.kexp16 = kexp16;
  pk.Q = Q;
  pk.wave = g.wave_d;
  (void)hipGetLastError();   // drop a stale code from an unrelated earlier HIP call of this thread
  hipError_t e = launch_pack(g, pk, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete L;
    return fail(SPS_E_HIP, "library packing failed: %s", hipGetErrorString(e));
  }
  tmp.release();
  const sps_status st = static_scratch_init(d->device);
  if (st != SPS_OK) {
    delete L;
    return st;
  }
  *out = L;
  return SPS_OK;
}

extern "C" sps_status sps_library_info_get(const sps_library *L, sps_library_info *o) {
  if (!L || !o) return fail(SPS_E_INVAL, "NULL argument");
  o->K = L->dev.K;
  o->K_pad = L->dev.K_pad;
  o->K_young_pad = L->dev.K_young_pad;
  o->N = L->dev.N;
  o->N_pad = L->dev.N_pad;
  o->n_young = L->n_young;
  o->n_line = L->n_line;
  o->device_bytes = L->mem.bytes;
  return SPS_OK;
}

extern "C" void sps_library_destroy(sps_library *L) {
  if (!L) return;
  if (L->device >= 0) (void)hipSetDevice(L->device);
  delete L;
}

extern "C" sps_status sps_theta_layout(const sps_library *L, sps_layout *o) {
  if (!L || !o) return fail(SPS_E_INVAL, "NULL argument");
  o->n_scalar = TH_NSCALAR;
  o->sfh = TH_NSCALAR;
  o->n_sfh = L->n_sfh;
  o->zh = TH_NSCALAR + L->n_sfh;
  o->n_zh = L->n_zh;
  o->P = L->dev.P;
  o->logmass = TH_LOGMASS;
  o->zred = TH_ZRED;
  o->tau_bc = TH_TAU_BC;
  o->alpha_bc = TH_ALPHA_BC;
  o->tau_diff = TH_TAU_DIFF;
  o->delta = TH_DELTA;
  o->logzsol = TH_LOGZSOL;
  o->gas_logz = TH_GAS_LOGZ;
  o->gas_logu = TH_GAS_LOGU;
  o->afe = TH_AFE;
  o->log_err_scale = TH_LOG_ERR_SCALE;
  o->log_f_calib = TH_LOG_F_CALIB;
  o->log_f_data = TH_LOG_F_DATA;
  o->log_jitter = TH_LOG_JITTER;
  o->frac_obrun = L->dev.escape ? L->dev.th_fob : -1;
  o->igm_factor = L->dev.igm ? L->dev.th_igm : -1;
  o->sigma_gal = L->dev.vdisp ? L->dev.th_sgal : -1;
  o->x_hi = (L->dev.igm & 2) ? L->dev.th_xhi : -1;
  o->log_nhi = (L->dev.igm & 4) ? L->dev.th_nhi : -1;
  o->z_dla = (L->dev.igm & 4) ? L->dev.th_nhi + 1 : -1;
  return SPS_OK;
}

// =====================================================================================
// Observations
// =====================================================================================
namespace sps {

static double sigma_inst_host(int mode, double v, double lam) {
  const double f = 2.3548200450309493;
  switch (mode) {
    case SPS_LSF_R_FWHM: return kC_kms / (f * v);
    case SPS_LSF_R_SIGMA: return kC_kms / v;
    case SPS_LSF_FWHM_AA: return kC_kms * v / (f * lam);
    case SPS_LSF_SIGMA_AA: return kC_kms * v / lam;
    case SPS_LSF_SIGMA_KMS: return v;
    default: return v / f;
  }
}

sps_status build_obs_operators(const sps_library *L, const sps_obs_desc *d, ObsHost &h, uint32_t *warnings) {
  if (warnings) *warnings = 0;
  double vd_ksig_kms_max = 0.0;   // widest continuum kernel of a spectrum (km/s)
  h.kind = d->kind;
  if (d->kind == SPS_OBS_PHOT) {
    if (d->n_band < 1 || d->n_band > 256) return fail(SPS_E_SHAPE, "n_band must be in [1, 256]");
    {
      long tot = 0;
      for (int b = 0; d->filter_len && b < d->n_band; ++b) tot += d->filter_len[b];
      if (tot > 4096) return fail(SPS_E_SHAPE, "at most 4096 filter nodes per observation");
    }
    if (!d->filter_len || !d->filter_wave || !d->filter_trans) return fail(SPS_E_INVAL, "filter arrays are NULL");
    h.n_data = d->n_band;
    h.band_off.assign(1, 0);
    size_t off = 0;
    for (int b = 0; b < d->n_band; ++b) {
      const int n = d->filter_len[b];
      if (n < 2) return fail(SPS_E_SHAPE, "filter %d has fewer than 2 nodes", b);
      const double *lam = d->filter_wave + off, *R = d->filter_trans + off;
      if (!finite_all(lam, n) || !increasing(lam, n) || lam[0] <= 0)
        return fail(SPS_E_INVAL, "filter %d wavelengths must be positive and increasing", b);
      for (int j = 0; j < n; ++j)
        if (!std::isfinite(R[j]) || R[j] < 0) return fail(SPS_E_INVAL, "filter %d transmission invalid", b);
      // eq. E1: numerator R lambda dlambda (central differences, one-sided ends);
      // zero point: trapezoid of R lambda f_lambda^AB
      double zp = 0.0;
      std::vector<double> num(n);
      for (int j = 0; j < n; ++j) {
        const double dl = j == 0 ? lam[1] - lam[0] : j == n - 1 ? lam[n - 1] - lam[n - 2] : 0.5 * (lam[j + 1] - lam[j - 1]);
        const double tw = j == 0 ? 0.5 * (lam[1] - lam[0]) : j == n - 1 ? 0.5 * (lam[n - 1] - lam[n - 2])
                                                                         : 0.5 * (lam[j + 1] - lam[j - 1]);
        const double fab = kFnuAB * kC_cms / ((lam[j] * kAng_cm) * (lam[j] * kAng_cm));
        zp += R[j] * lam[j] * tw * fab;
        num[j] = R[j] * lam[j] * dl;
      }
      if (!(zp > 0)) return fail(SPS_E_INVAL, "filter %d has zero transmission", b);
      for (int j = 0; j < n; ++j) {
        h.fw.push_back(lam[j]);
        h.fwln.push_back(std::log(lam[j]));
        h.fr.push_back(num[j] / zp);
        h.fr_f.push_back((float)(num[j] / zp));
      }
      off += n;
      h.band_off.push_back((int)off);
    }
  } else if (d->kind == SPS_OBS_SPEC) {
    const int np = d->n_pix;
    if (np < 2) return fail(SPS_E_SHAPE, "n_pix must be >= 2");
    if (!d->pix_wave || !finite_all(d->pix_wave, np) || !increasing(d->pix_wave, np) || d->pix_wave[0] <= 0)
      return fail(SPS_E_INVAL, "pixel wavelengths must be positive and increasing");
    if (d->lsf_mode == SPS_LSF_BARE_R)
      return fail(SPS_E_INVAL, "a bare resolving power is ambiguous: state R_fwhm or R_sigma (App. F)");
    if (d->lsf_mode < 0 || d->lsf_mode > SPS_LSF_FWHM_KMS) return fail(SPS_E_INVAL, "unknown LSF mode %d", d->lsf_mode);
    if (!d->lsf_curve && !(d->lsf_value > 0)) return fail(SPS_E_INVAL, "LSF value must be > 0");
    if (d->lsf_curve)
      for (int i = 0; i < np; ++i)
        if (!(d->lsf_curve[i] > 0) || !std::isfinite(d->lsf_curve[i])) return fail(SPS_E_INVAL, "LSF curve must be > 0");
    if (!(d->z_ref >= 0) || !(d->sigma_gal_kms >= 0) || !(d->sigma_gas_kms >= 0))
      return fail(SPS_E_INVAL, "z_ref and dispersions must be >= 0");
    h.n_data = np;
    h.pix.assign(d->pix_wave, d->pix_wave + np);
    h.lnpix.resize(np);
    h.ksig.resize(np);
    // library resolution floor (eq. F3): (c / 2.3548) * 2 dlambda / lambda on the stored grid
    const int N = L->dev.N;
    std::vector<double> lw(N), slib(N);
    L->host_wave(lw);
    for (int n = 0; n < N; ++n) {
      const double dl = n == 0 ? lw[1] - lw[0] : n == N - 1 ? lw[N - 1] - lw[N - 2] : 0.5 * (lw[n + 1] - lw[n - 1]);
      slib[n] = kC_kms / 2.3548200450309493 * 2.0 * dl / lw[n];
    }
    int finer = 0;
    for (int i = 0; i < np; ++i) {
      const double lam = d->pix_wave[i];
      h.lnpix[i] = std::log(lam);
      const double v = d->lsf_curve ? d->lsf_curve[i] : d->lsf_value;
      const double si = sigma_inst_host(d->lsf_mode, v, lam);
      const double lr = lam / (1.0 + d->z_ref);
      double sl;
      if (lr <= lw[0]) sl = slib[0];
      else if (lr >= lw[N - 1]) sl = slib[N - 1];
      else {
        const int j = (int)(std::upper_bound(lw.begin(), lw.end(), lr) - lw.begin()) - 1;
        sl = slib[j] + (lr - lw[j]) / (lw[j + 1] - lw[j]) * (slib[j + 1] - slib[j]);
      }
      if (si < sl) ++finer;
      const double sfix2 = std::max(si * si - sl * sl, 0.0);
      const double sk = std::sqrt(sfix2 + d->sigma_gal_kms * d->sigma_gal_kms);
      vd_ksig_kms_max = std::max(vd_ksig_kms_max, sk);
      h.ksig[i] = sk / kC_kms;
    }
    if (finer && warnings) *warnings |= SPS_WARN_LSF_FINER_THAN_LIBRARY;
    h.lsf_mode = d->lsf_mode;
    h.lsf_value = d->lsf_value;
    if (d->lsf_curve) h.lsf_vals.assign(d->lsf_curve, d->lsf_curve + np);
    h.sigma_gas = d->sigma_gas_kms;
    // calibration polynomial (Sec. 3.2, App. H.3): x maps the first pixel to -1, the last to +1
    if (d->calib_mode < SPS_CALIB_NONE || d->calib_mode > SPS_CALIB_OPTIMISE)
      return fail(SPS_E_INVAL, "unknown calibration mode %d", d->calib_mode);
    h.calib_mode = d->calib_mode;
    if (d->calib_mode != SPS_CALIB_NONE) {
      if (d->calib_order < 0 || d->calib_order > 7) return fail(SPS_E_SHAPE, "calib_order must be in [0, 7]");
      if (!d->calib_prior) return fail(SPS_E_INVAL, "calib_prior is NULL");
      for (int m = 0; m <= d->calib_order; ++m)
        if (!(d->calib_prior[m] > 0) || !std::isfinite(d->calib_prior[m]))
          return fail(SPS_E_INVAL, "calibration prior widths must be finite and > 0");
      h.calib_order = d->calib_order;
      h.calib_prior.assign(d->calib_prior, d->calib_prior + d->calib_order + 1);
      h.calib_xs = 2.0 / (d->pix_wave[np - 1] - d->pix_wave[0]);
      h.calib_x0 = -1.0 - d->pix_wave[0] * h.calib_xs;
    }
    // analytic marginalisation of the line fluxes (Sec. 4.1, App. I.3)
    if (d->line_marg < SPS_LINEMARG_NONE || d->line_marg > SPS_LINEMARG_FLAT)
      return fail(SPS_E_INVAL, "unknown line_marg mode %d", d->line_marg);
    h.lm_mode = d->line_marg;
    if (h.lm_mode != SPS_LINEMARG_NONE) {
      const int nl = L->n_line;
      if (nl < 1) return fail(SPS_E_INVAL, "line marginalisation needs a library with nebular lines");
      if (h.calib_mode != SPS_CALIB_NONE)
        return fail(SPS_E_INVAL, "line marginalisation and a calibration polynomial together are not supported");
      if (np > 8192) return fail(SPS_E_SHAPE, "line marginalisation takes spectra of at most 8192 pixels");
      if (h.lm_mode == SPS_LINEMARG_GAUSS && !(d->line_prior_frac > 0 && std::isfinite(d->line_prior_frac)))
        return fail(SPS_E_INVAL, "line_prior_frac must be finite and > 0");
      h.lm_frac = d->line_prior_frac;
      if (d->line_flat) {
        h.lm_flat.resize(nl);
        for (int l = 0; l < nl; ++l) h.lm_flat[l] = d->line_flat[l] ? 1 : 0;
      }
      // at most kLineMargMax lines in any rest interval as wide as the pixel range (ln)
      const double width = std::log(d->pix_wave[np - 1] / d->pix_wave[0]);
      int most = 0;
      for (int l0 = 0, l1 = 0; l0 < nl; ++l0) {
        while (l1 < nl && std::log(L->line_wave_h[l1] / L->line_wave_h[l0]) <= width) ++l1;
        most = std::max(most, l1 - l0);
      }
      if (most > kLineMargMax)
        return fail(SPS_E_SHAPE, "up to %d library lines fall within the pixel range; the marginalisation fits at "
                    "most %d", most, kLineMargMax);
      h.lm_most = most;
    }
  } else if (d->kind == SPS_OBS_LINES) {
    // emission-line catalogue (Sec. 3.3, App. I): blends of the library's lines
    const int nk = d->n_band;
    if (L->n_line < 1) return fail(SPS_E_INVAL, "a line catalogue needs a library with nebular lines");
    if (nk < 1 || nk > 4096) return fail(SPS_E_SHAPE, "a line catalogue holds 1 to 4096 entries");
    if (!d->line_len || !d->line_index) return fail(SPS_E_INVAL, "line_len / line_index are NULL");
    h.n_data = nk;
    h.loff.assign(1, 0);
    for (int k = 0; k < nk; ++k) {
      const int n = d->line_len[k];
      if (n < 1 || n > L->n_line) return fail(SPS_E_SHAPE, "catalogue entry %d: blend of %d lines", k, n);
      for (int j = 0; j < n; ++j) {
        const int l = d->line_index[h.loff.back() + j];
        if (l < 0 || l >= L->n_line) return fail(SPS_E_INVAL, "catalogue entry %d: line index %d", k, l);
        for (int q = h.loff.back(); q < (int)h.lidx.size(); ++q)
          if (h.lidx[q] == l) return fail(SPS_E_INVAL, "catalogue entry %d: line %d listed twice", k, l);
        h.lidx.push_back(l);
      }
      h.loff.push_back(h.loff.back() + n);
    }
    h.upper.assign(nk, 0);
    if (d->upper)
      for (int k = 0; k < nk; ++k) h.upper[k] = d->upper[k] ? 1 : 0;
  } else {
    return fail(SPS_E_INVAL, "unknown observation kind %d", d->kind);
  }
  h.noise_flags = d->noise_flags & 15u;
  if (L->dev.vdisp && (h.kind == SPS_OBS_PHOT || h.kind == SPS_OBS_SPEC)) {
    // Fourier stage of a free sigma_gal (Sec. 2.5, App. F): the observed range whose rest
    // frame the projection reads, the window margin M in nodes (the banded rows' reach,
    // sigma_max's reach, the interpolation brackets) and the power-of-two transform length
    // that holds the longest window plus sigma_max's reach on each side
    const double dlnl = L->dev.dlnw;
    const int mg = (int)std::ceil(5.0 * L->dev.vd_max / (kC_kms * dlnl));
    double lo, hi;
    int M;
    if (h.kind == SPS_OBS_SPEC) {
      lo = h.pix.front();
      hi = h.pix.back();
      M = (int)std::ceil(5.0 * vd_ksig_kms_max / (kC_kms * dlnl)) + mg + 2;
    } else {
      lo = *std::min_element(h.fw.begin(), h.fw.end());
      hi = *std::max_element(h.fw.begin(), h.fw.end());
      M = mg + 2;
    }
    const double need = std::ceil(std::log(hi / lo) / dlnl) + 2.0 * M + 2.0 + 2.0 * mg;
    int n = 1, lg = 0;
    while (n < need && n <= kVdispMaxFFT) {
      n *= 2;
      ++lg;
    }
    if (n > kVdispMaxFFT)
      return fail(SPS_E_SHAPE, "the Fourier stage of this observation needs a transform of %.0f points (at most %d)",
                  need, kVdispMaxFFT);
    h.vd_M = M;
    h.vd_nfft = n;
    h.vd_log2 = lg;
    h.vd_lnlo = std::log(lo);
    h.vd_lnhi = std::log(hi);
    h.vd_dlnl = dlnl;
    h.vd_tw.resize((size_t)n);
    for (int k = 0; k < n / 2; ++k) {
      h.vd_tw[2 * k] = std::cos(2.0 * kPi * k / n);
      h.vd_tw[2 * k + 1] = -std::sin(2.0 * kPi * k / n);
    }
  }
  return SPS_OK;
}

sps_status set_obs_data(ObsHost &h, const double *data, const double *sigma, const uint8_t *mask) {
  const int n = h.n_data;
  h.data.assign(n, 0.0);
  h.sigma.assign(n, 1.0);
  h.mask.assign(n, 0);
  h.ivar.assign(n, 0.0);
  h.lnorm = 0.0;
  if (!data || !sigma) return SPS_OK;   // no data: logL over an empty mask is 0
  for (int i = 0; i < n; ++i) {
    const bool ok = std::isfinite(data[i]) && std::isfinite(sigma[i]) && sigma[i] > 0 && (!mask || mask[i]);
    h.mask[i] = ok ? 1 : 0;
    if (ok) {
      h.data[i] = data[i];
      h.sigma[i] = sigma[i];
      h.ivar[i] = 1.0 / (sigma[i] * sigma[i]);
      h.lnorm -= 0.5 * std::log(2.0 * M_PI * sigma[i] * sigma[i]);
    }
  }
  return SPS_OK;
}

}  // namespace sps

extern "C" sps_status sps_obs_create(const sps_library *L, const sps_obs_desc *d, sps_obs **out, uint32_t *warnings) {
  if (!L || !d || !out) return fail(SPS_E_INVAL, "sps_obs_create: NULL argument");
  *out = nullptr;
  if (L->device < 0) return fail(SPS_E_STATE, "host-only library: observations need a device library");
  if (d->max_batch < 1 || d->max_batch > (1 << 20)) return fail(SPS_E_SHAPE, "max_batch must be in [1, 2^20]");
  if (hipSetDevice(L->device) != hipSuccess) return fail(SPS_E_HIP, "hipSetDevice failed");
  auto *o = new sps_obs();
  o->lib = L;
  sps_status st = build_obs_operators(L, d, o->host, warnings);
  if (st == SPS_OK) st = set_obs_data(o->host, d->data, d->sigma, d->mask);
  if (st == SPS_OK) st = o->upload_operators();
  if (st == SPS_OK) st = o->ws.create(L, d->max_batch, o->host.n_data, (int)o->host.fw.size());
  if (st != SPS_OK) {
    delete o;
    return st;
  }
  *out = o;
  return SPS_OK;
}

extern "C" sps_status sps_obs_set_data(sps_obs *o, const double *data, const double *sigma, const uint8_t *mask) {
  if (!o) return fail(SPS_E_INVAL, "NULL observation");
  if (hipSetDevice(o->lib->device) != hipSuccess) return fail(SPS_E_HIP, "hipSetDevice failed");
  sps_status st = set_obs_data(o->host, data, sigma, mask);
  if (st != SPS_OK) return st;
  return o->upload_data();
}

extern "C" int32_t sps_obs_n_data(const sps_obs *o) { return o ? o->host.n_data : -1; }

extern "C" void sps_obs_destroy(sps_obs *o) {
  if (!o) return;
  (void)hipSetDevice(o->lib->device);
  delete o;
}

// =====================================================================================
// Hot calls
// =====================================================================================
namespace sps {

bool precision_built(const sps_library *L, int p) { return p >= 0 && p <= 9 && (L->precisions >> p) & 1u; }

sps_status launch_forward(const sps_library *L, Workspace &w, const DevObs *obs_table, const int *point_obs,
                          const double *theta, int B, int prec, double *logl, double *model, int ld_model,
                          bool grad, int ld_g, const ObsHost *one, sps_obs *timing_obs, hipStream_t s,
                          bool keep_sorted_model, const LineMargLaunch *joint) {
  if (B < 1 || B > w.max_batch) return fail(SPS_E_SHAPE, "B=%d outside [1, max_batch=%d]", B, w.max_batch);
  if (!precision_built(L, prec)) return fail(SPS_E_INVAL, "precision %d not built into this library", prec);
  const DevLib &g = L->dev;
  if (g.vdisp && !one) return fail(SPS_E_INVAL, "a free sigma_gal needs a single observation per launch");
  const int B_pad = (B + kMAlign - 1) / kMAlign * kMAlign;
  // the thread's HIP last-error slot may hold a stale code set by another library's
  // call; clear it so that only this call's own launches are checked below
  (void)hipGetLastError();
  const int mode = prec == 0 ? 0 : prec == 1 ? 1 : (prec == 2 || prec == 4 || prec == 6 || prec == 8) ? 2 : 3;
  const int MT = contract_mtile(prec, B_pad);
  const int tf = contract_ktile_factor(prec);
  int *ranks = B >= kRankKernelMinB ? w.ranks : nullptr;
  hipError_t e = launch_keys(g, theta, g.P, B, w.keys, ranks, s);
  PrepLaunch pl;
  pl.theta = theta;
  pl.P = g.P;
  pl.B = B;
  pl.B_pad = B_pad;
  pl.keys = B <= kSelfKeyMaxB ? nullptr : w.keys;   // NULL: the weight builder forms the keys
  pl.ranks = ranks;
  pl.obs_table = obs_table;
  pl.point_obs = point_obs;
  pl.W = w.W;
  pl.Wlo = (char *)w.W + (size_t)B_pad * g.K_pad * 2;
  pl.rowmask = w.rowmask;
  pl.mask_words = w.mask_words;
  pl.rows = w.rows;
  pl.Lline = w.Lline;
  pl.WQ = g.has_cont ? w.WQ : nullptr;
  pl.kpos = L->kpos_d;
  pl.line_k0 = L->line_k0;
  pl.mode = mode;
  if (g.has_cont && !w.WQ) return fail(SPS_E_STATE, "workspace has no nebular-continuum buffer");
  if (e == hipSuccess) e = launch_prep(g, pl, s);
  // launches on a log-uniform grid compute only the tiles whose pixels the projection reads
  // (the rows' spans); so does the gradient pass, whose attenuation adjoint reads F and the
  // young part only where d logL / d F can be nonzero; the FP64 instance stays dense
  // the single-observation path knows its observation: a line catalogue needs no rest-frame
  // spectrum (no contraction), a calibration polynomial the model at the sorted rows and a
  // pass of its own after the projection
  const bool lines_only = one && one->kind == SPS_OBS_LINES;
  const bool calib = one && one->calib_mode != SPS_CALIB_NONE;
  const bool lmarg = one && one->lm_mode != SPS_LINEMARG_NONE;
  if ((calib || lmarg) && (grad || !w.mbuf || !w.scr || w.ld_scr < std::max(24, 2 * one->n_data)))
    return fail(SPS_E_INVAL, "calibration polynomial / line marginalisation: no gradient, and a full workspace");
  const int n_nt = g.N_pad / 64;
  const bool dense_small = !grad && B_pad <= kDenseMaxBpad && (B_pad / MT) * n_nt <= kDenseMaxBlocks;
  const bool span = g.log_uniform && prec != SPS_FP64 && w.tiles && B_pad / MT <= kTileListMaxM && !dense_small;
  w.f_spans = span && !lines_only;
  ContractLaunch cl;
  cl.list = span ? w.tiles : nullptr;
  if (span && !lines_only && e == hipSuccess) e = launch_tile_list(w.rows, B_pad, MT, n_nt, prec != SPS_FP32, w.tiles, s);
  cl.W = pl.W;
  cl.Wlo = pl.Wlo;
  cl.B_pad = B_pad;
  cl.rowmask = w.rowmask;
  cl.mask_words = w.mask_words;
  cl.counter = w.counter;
  cl.rows = w.rows;
  cl.F = w.F;
  cl.Yatt = grad ? w.Yatt : nullptr;
  cl.precision = prec;
  cl.pass = 0;
  cl.ev_start = cl.ev_stop = nullptr;
  if (e == hipSuccess && timing_obs && !lines_only)
    e = timing_obs->timing_events((B_pad / MT) * n_nt, g.K_pad / (kKTile * tf), &cl.ev_start, &cl.ev_stop);
  if (e == hipSuccess && !lines_only) e = launch_contract(g, cl, s);
  if (g.escape == SPS_ESCAPE_PICKET && !lines_only && e == hipSuccess) {
    // the picket fence's dust-free part: f_ob (young stars + ionising continuum), added to F
    ContractLaunch c1 = cl;
    c1.pass = 1;
    c1.ev_start = c1.ev_stop = nullptr;
    e = launch_contract(g, c1, s);
  }
  if (g.has_cont && !lines_only && e == hipSuccess) {
    NebLaunch nb;
    nb.theta = theta;
    nb.rows = w.rows;
    nb.WQ = w.WQ;
    nb.F = w.F;
    nb.list = cl.list;
    nb.B_pad = B_pad;
    nb.MT = cl.list ? MT : 64;
    nb.f64 = prec == SPS_FP64;
    e = launch_nebular(g, nb, s);
  }
  if (g.vdisp && one->vd_nfft > 0 && e == hipSuccess) {
    // the Fourier stage of a free sigma_gal, before the projection (which applies the IGM)
    VdispLaunch vl;
    vl.obs = obs_table;
    vl.theta = theta;
    vl.rows = w.rows;
    vl.F = w.F;
    vl.B_pad = B_pad;
    vl.nfft = one->vd_nfft;
    vl.log2n = one->vd_log2;
    vl.f64 = prec == SPS_FP64;
    e = launch_vdisp(g, vl, s);
  }
  ProjectLaunch pj;
  pj.obs_table = obs_table;
  pj.rows = w.rows;
  pj.F = w.F;
  pj.f64 = prec == 0;
  pj.theta = theta;
  pj.P = g.P;
  pj.B = B;
  pj.Lline = w.Lline;
  pj.model = model;
  pj.logl = logl;
  pj.gvec = grad ? w.gvec : nullptr;
  pj.gnoise = grad ? w.gnoise : nullptr;
  pj.msorted = grad || calib || lmarg || keep_sorted_model ? w.mbuf : nullptr;
  pj.ld_model = ld_model;
  pj.ld_g = ld_g;
  if (e == hipSuccess) e = launch_project(g, pj, s);
  if (calib && e == hipSuccess) {
    CalibLaunch cb;
    cb.obs_table = obs_table;
    cb.rows = w.rows;
    cb.theta = theta;
    cb.msorted = w.mbuf;
    cb.ld = ld_g;
    cb.B_pad = B_pad;
    cb.sums = w.scr;
    cb.ld_sums = w.ld_scr;
    cb.logl = logl;
    e = launch_calib(g, cb, s);
  }
  if (lmarg && e == hipSuccess) {
    LineMargLaunch lm;
    lm.obs_table = obs_table;
    lm.rows = w.rows;
    lm.theta = theta;
    lm.Lline = w.Lline;
    lm.msorted = w.mbuf;
    lm.ld = ld_g;
    lm.scr = w.scr;
    lm.ld_scr = w.ld_scr;
    lm.B_pad = B_pad;
    lm.logl = logl;
    lm.cat = joint ? joint->cat : nullptr;
    lm.cat_model = joint ? joint->cat_model : nullptr;
    lm.cat_ld = joint ? joint->cat_ld : 0;
    lm.phot = joint ? joint->phot : nullptr;
    lm.phot_model = joint ? joint->phot_model : nullptr;
    lm.phot_ld = joint ? joint->phot_ld : 0;
    lm.phot_scr = joint ? joint->phot_scr : nullptr;
    lm.phot_ld_scr = joint ? joint->phot_ld_scr : 0;
    lm.lprof = joint ? joint->lprof : nullptr;
    lm.lprof_k0 = joint ? joint->lprof_k0 : nullptr;
    lm.lprof_len = joint ? joint->lprof_len : nullptr;
    lm.lprof_w = joint ? joint->lprof_w : 0;
    e = launch_linemarg(g, lm, s);
  }
  if (e != hipSuccess) return fail(SPS_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return SPS_OK;
}

sps_status run_forward(const sps_library *L, sps_obs *o, const double *theta, int B, int prec, double *logl,
                       double *model, bool want_grad_buffers, hipStream_t s) {
  if (!L || !o || !theta) return fail(SPS_E_INVAL, "NULL argument");
  if (o->lib != L) return fail(SPS_E_INVAL, "observation belongs to another library");
  return launch_forward(L, o->ws, o->dev_obs, nullptr, theta, B, prec, logl, model, o->host.n_data,
                        want_grad_buffers, o->host.n_data, &o->host, o, s);
}

}  // namespace sps

extern "C" sps_status sps_forward(const sps_library *L, sps_obs *o, const double *theta, int32_t B, int32_t prec,
                                  double *model, void *stream) {
  if (!model) return fail(SPS_E_INVAL, "model_dev is NULL");
  return run_forward(L, o, theta, B, prec, nullptr, model, false, (hipStream_t)stream);
}

extern "C" sps_status sps_logl(const sps_library *L, sps_obs *o, const double *theta, int32_t B, int32_t prec,
                               double *logl, double *model, void *stream) {
  if (!logl) return fail(SPS_E_INVAL, "logl_dev is NULL");
  return run_forward(L, o, theta, B, prec, logl, model, false, (hipStream_t)stream);
}

extern "C" sps_status sps_logl_grad(const sps_library *L, sps_obs *o, const double *theta, int32_t B, int32_t prec,
                                    double *logl, double *grad, void *stream) {
  if (!logl || !grad) return fail(SPS_E_INVAL, "logl_dev / grad_dev is NULL");
  if (prec != SPS_FP64 && prec != SPS_FP32) return fail(SPS_E_INVAL, "gradients are available for FP64 and FP32");
  if (o && (o->host.kind == SPS_OBS_LINES || o->host.calib_mode != SPS_CALIB_NONE ||
            o->host.lm_mode != SPS_LINEMARG_NONE))
    return fail(SPS_E_INVAL, "gradients are not available for line catalogues, calibrated spectra or marginalised "
                "line fluxes");
  if (L && (L->dev.has_cont || L->dev.escape || L->line_tau_axis || L->dev.sfh_scheme || L->dev.igm || L->dev.vdisp))
    return fail(SPS_E_INVAL, "gradients are not available for libraries with a nebular continuum cube, an escape "
                "geometry, a line table on an age axis of its own, the linear SFH scheme, the IGM or a free "
                "sigma_gal");
  sps_status st = run_forward(L, o, theta, B, prec, logl, nullptr, true, (hipStream_t)stream);
  if (st != SPS_OK) return st;
  return run_adjoint(L, o, theta, B, prec, grad, (hipStream_t)stream);
}

extern "C" sps_status sps_logl_lines_joint(const sps_library *L, sps_obs *spec, sps_obs *cat, sps_obs *phot,
                                           const double *theta, int32_t B, int32_t prec, double *logl, void *stream) {
  if (!L || !spec || !theta || !logl) return fail(SPS_E_INVAL, "NULL argument");
  if (spec->lib != L || (cat && cat->lib != L) || (phot && phot->lib != L))
    return fail(SPS_E_INVAL, "observation belongs to another library");
  if (spec->host.kind != SPS_OBS_SPEC || spec->host.lm_mode == SPS_LINEMARG_NONE ||
      (cat && cat->host.kind != SPS_OBS_LINES) || (phot && phot->host.kind != SPS_OBS_PHOT))
    return fail(SPS_E_INVAL, "a joint marginalisation takes a spectrum with line_marg set, a line catalogue and a "
                "photometric observation (each of the last two may be NULL)");
  int n_cat = 0;
  if (cat) {
    if (cat->host.n_data > kLineCatMaxHost)
      return fail(SPS_E_SHAPE, "a jointly marginalised catalogue holds at most %d entries", kLineCatMaxHost);
    std::vector<uint8_t> seen(L->n_line, 0);
    for (int l : cat->host.lidx) n_cat += seen[l] ? 0 : (seen[l] = 1);
  }
  if (spec->host.lm_most + n_cat > kLineMargMax)
    return fail(SPS_E_SHAPE, "up to %d lines would be fitted jointly; at most %d", spec->host.lm_most + n_cat,
                kLineMargMax);
  if (phot) {
    if (L->dev.vdisp)
      return fail(SPS_E_INVAL, "a joint marginalisation with photometry takes a library without a free sigma_gal");
    if (!L->lprof_d || (size_t)phot->ws.ld_scr < (size_t)phot->host.n_data * (kLineMargMax + 2))
      return fail(SPS_E_SHAPE, "the photometric observation's scratch holds no band responses (%d bands)",
                  phot->host.n_data);
  }
  if (L->dev.vdisp && (spec->host.vd_nfft <= 0)) return fail(SPS_E_STATE, "spectrum without its Fourier plan");
  hipStream_t s = (hipStream_t)stream;
  // the catalogue and the photometry first (their logL land in logl and are replaced),
  // their models kept at the sorted rows; the spectrum's rows come in the same order
  // (same points, same keys)
  sps_status st = SPS_OK;
  if (cat)
    st = launch_forward(L, cat->ws, cat->dev_obs, nullptr, theta, B, prec, logl, nullptr, cat->host.n_data, false,
                        cat->host.n_data, &cat->host, nullptr, s, true, nullptr);
  if (st == SPS_OK && phot)
    st = launch_forward(L, phot->ws, phot->dev_obs, nullptr, theta, B, prec, logl, nullptr, phot->host.n_data,
                        false, phot->host.n_data, &phot->host, nullptr, s, true, nullptr);
  if (st != SPS_OK) return st;
  LineMargLaunch j{};
  j.cat = cat ? cat->dev_obs : nullptr;
  j.cat_model = cat ? cat->ws.mbuf : nullptr;
  j.cat_ld = cat ? cat->host.n_data : 0;
  j.phot = phot ? phot->dev_obs : nullptr;
  j.phot_model = phot ? phot->ws.mbuf : nullptr;
  j.phot_ld = phot ? phot->host.n_data : 0;
  j.phot_scr = phot ? phot->ws.scr : nullptr;
  j.phot_ld_scr = phot ? phot->ws.ld_scr : 0;
  j.lprof = L->lprof_d;
  j.lprof_k0 = L->lprof_k0_d;
  j.lprof_len = L->lprof_len_d;
  j.lprof_w = L->lprof_w;
  return launch_forward(L, spec->ws, spec->dev_obs, nullptr, theta, B, prec, logl, nullptr, spec->host.n_data, false,
                        spec->host.n_data, &spec->host, spec, s, false, &j);
}

extern "C" sps_status sps_obs_enable_timing(sps_obs *o, int32_t enable) {
  if (!o) return fail(SPS_E_INVAL, "NULL observation");
  return o->enable_timing(enable != 0);
}

extern "C" sps_status sps_obs_contract_timing(sps_obs *o, double *ms, int64_t *launches, int64_t *exec_tiles,
                                              int64_t *dense_tiles) {
  if (!o) return fail(SPS_E_INVAL, "NULL observation");
  return o->read_timing(ms, launches, exec_tiles, dense_tiles);
}

extern "C" const char *sps_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *sps_version(void) { return "sps-gfx950 0.1"; }
