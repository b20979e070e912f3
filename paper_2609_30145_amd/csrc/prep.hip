// Per-point preparation: batch ordering, cosmology, SFH x ZH -> SSP weights, nebular
// line luminosities and the K-tile occupancy of the contraction.
#include "common.h"
#include "kernels.h"

namespace sps {

// ---------------------------------------------------------------------------------
// Batch ordering.  Rows that share a redshift (time-varying enrichment) or a
// metallicity/alpha bracket (constant metallicity) are grouped so that whole
// K tiles of the weight matrix are zero for an M tile and can be skipped.
// ---------------------------------------------------------------------------------
__device__ double sort_key(const DevLib &lib, const double *th) {
  double z = th[TH_ZRED];
  if (lib.n_zh > 0) return z;
  int jz = 0;
  double t;
  bool in;
  if (lib.n_z > 1) grid_split_dev(lib.logz, lib.n_z, th[TH_LOGZSOL], jz, t, in);
  int ja = 0;
  if (lib.n_afe > 1) grid_split_dev(lib.afe, lib.n_afe, th[TH_AFE], ja, t, in);
  return (double)jz * 1.0e6 + (double)ja * 1.0e4 + fmin(fmax(z, 0.0), 9.0e3);
}

__global__ void __launch_bounds__(256) k_keys(DevLib lib, const double *__restrict__ theta, int P, int B,
                                              double *__restrict__ keys) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b < B) keys[b] = sort_key(lib, theta + (size_t)b * P);
}

// One workgroup per point: rank = number of points with a smaller (key, index).
__global__ void __launch_bounds__(256) k_sort(const double *__restrict__ keys, int B, int *__restrict__ perm) {
  __shared__ int cnt[256];
  const int b = blockIdx.x;
  const double my = keys[b];
  int c = 0;
  for (int j = threadIdx.x; j < B; j += 256) {
    const double kj = keys[j];
    c += (kj < my) || (kj == my && j < b);
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) perm[cnt[0]] = b;
}

// ---------------------------------------------------------------------------------
// Weight builder.  One workgroup per sorted row.
// ---------------------------------------------------------------------------------
template <int NT>
__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ double block_max(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return *reinterpret_cast<uint16_t *>(&h);
}
__device__ __forceinline__ float f16_to_f(uint16_t h) {
  _Float16 v = *reinterpret_cast<_Float16 *>(&h);
  return (float)v;
}

// Output mode of the weight row.
enum WMode { W_F64 = 0, W_F32 = 1, W_BF16 = 2, W_F16 = 3 };

struct PrepArgs {
  const double *theta;
  int P, B, B_pad;
  const int *perm;
  const DevObs *obs_table;
  const int *point_obs;     // [B] observation slot per point, NULL = slot 0
  void *W;                  // F64/F32: [B_pad][K_pad]; 16-bit: hi plane
  void *Wlo;                // 16-bit residual plane
  uint32_t *rowmask;        // [B_pad][mask_words]
  int mask_words;
  PointRow *rows;           // [B_pad]
  double *Lline;            // [B_pad][n_line] (spectra: line luminosities, erg/s per Msun)
  const int *kpos;          // [n_afe][n_z][n_age] -> K position
  int line_k0;              // K position of line 0 (photometric path)
};

template <int MODE>
__global__ void __launch_bounds__(256) k_prep(DevLib lib, PrepArgs a) {
  extern __shared__ double smem[];
  const int K_pad = lib.K_pad;
  double *wacc = smem;                        // [K_pad]
  double *edges = wacc + K_pad;               // [n_sfh + 1]
  double *zt = edges + lib.n_sfh + 1;         // [n_sfh] fraction t
  int *zj = (int *)(zt + lib.n_sfh);          // [n_sfh] node j
  double *red = (double *)(zj + ((lib.n_sfh + 1) & ~1));   // [256]
  double *wq = red + 256;                     // [n_young]
  __shared__ double s_th[TH_NSCALAR];
  __shared__ double s_sc[4];

  const int r = blockIdx.x;
  const int tid = threadIdx.x;
  const int b = r < a.B ? a.perm[r] : -1;

  if (b < 0) {   // padding row: zero weights
    for (int k = tid; k < K_pad; k += 256) {
      if (MODE == W_F64) ((double *)a.W)[(size_t)r * K_pad + k] = 0.0;
      else if (MODE == W_F32) ((float *)a.W)[(size_t)r * K_pad + k] = 0.f;
      else {
        ((uint16_t *)a.W)[(size_t)r * K_pad + k] = 0;
        ((uint16_t *)a.Wlo)[(size_t)r * K_pad + k] = 0;
      }
    }
    for (int w = tid; w < a.mask_words; w += 256) a.rowmask[(size_t)r * a.mask_words + w] = 0u;
    if (tid == 0) {
      PointRow pr = {};
      pr.b = -1;
      a.rows[r] = pr;
    }
    return;
  }
  const double *th = a.theta + (size_t)b * a.P;
  if (tid < TH_NSCALAR) s_th[tid] = th[tid];
  for (int k = tid; k < K_pad; k += 256) wacc[k] = 0.0;
  __syncthreads();

  // ---- cosmology (Sec. 2.6): t_univ closed form; D_C by composite Gauss-Legendre in
  //      u = (1+z')^-1/2, where the integrand 2 / sqrt(Om + OL u^6) is smooth.
  const double z = s_th[TH_ZRED];
  const double Om = lib.Om, OL = 1.0 - lib.Om;
  const double tH_yr = kMpc_km / lib.H0 / kYr_s;
  const double DH_mpc = kC_kms / lib.H0;
  const double u0 = 1.0 / sqrt(1.0 + z);
  double part = 0.0;
  for (int i = tid; i < lib.n_gl; i += 256) {
    const double u = u0 + (1.0 - u0) * lib.gl_u[i];
    const double u2 = u * u;
    part += lib.gl_w[i] * 2.0 / sqrt(Om + OL * u2 * u2 * u2);
  }
  const double dc_int = block_sum<256>(part, red) * (1.0 - u0);
  if (tid == 0) {
    const double t_univ = tH_yr * 2.0 / (3.0 * sqrt(OL)) * asinh(sqrt(OL / Om) * pow(1.0 + z, -1.5));
    s_sc[0] = t_univ;
    s_sc[1] = DH_mpc * dc_int * kMpc_cm;    // D_C [cm]
  }
  __syncthreads();
  const double t_univ = s_sc[0];
  const double dc = s_sc[1];
  const double dl = (1.0 + z) * dc;

  // ---- SFH edges, rescaled to t_univ (App. B, Sec. 2.6)
  const int n_sfh = lib.n_sfh;
  const double lnR = log(t_univ / lib.T1);
  for (int i = tid; i <= n_sfh; i += 256) {
    double T;
    if (i == 0) T = 0.0;
    else if (i == 1) T = lib.T1;
    else if (i == n_sfh) T = t_univ;
    else T = lib.T1 * exp(lnR * (double)(i - 1) / (double)(n_sfh - 1));
    edges[i] = T;
  }
  // ---- per-bin metallicity and its bracketing nodes (Sec. 2.2.2)
  //      time-varying mode: nodes and bin centres are both log-uniform from T1 to
  //      t_univ, so the interpolation weight in ln T is fixed in the normalised
  //      coordinate: bin i >= 1 sits at (i - 1/2)/(n_sfh - 1), node k at k/(n_zh - 1);
  //      the first bin (centre T1/2) is clamped to node 0.
  const double *zh = th + TH_NSCALAR + n_sfh;
  for (int i = tid; i < n_sfh; i += 256) {
    double zeta;
    if (lib.n_zh == 0) {
      zeta = s_th[TH_LOGZSOL];
    } else if (i == 0 || lib.n_zh == 1) {
      zeta = zh[0];
    } else {
      const double x = ((double)i - 0.5) / (double)(n_sfh - 1) * (double)(lib.n_zh - 1);
      int k = (int)floor(x);
      if (k >= lib.n_zh - 1) k = lib.n_zh - 2;
      const double f = x - (double)k;
      zeta = zh[k] + f * (zh[k + 1] - zh[k]);
    }
    int j = 0;
    double t = 0.0;
    bool in;
    if (lib.n_z > 1) grid_split_dev(lib.logz, lib.n_z, zeta, j, t, in);
    zj[i] = j;
    zt[i] = t;
  }
  int ja = 0;
  double ta = 0.0;
  if (lib.n_afe > 1) {
    bool in;
    grid_split_dev(lib.afe, lib.n_afe, s_th[TH_AFE], ja, ta, in);
  }
  __syncthreads();

  // ---- step-scheme overlap weights (App. B): thread per SSP age node, so every
  //      (alpha, m, a) slot of the LDS row has a single writer.
  const double *mass = th + TH_NSCALAR;
  const int na = lib.n_age, nz = lib.n_z, nf = lib.n_afe;
  for (int ag = tid; ag < na; ag += 256) {
    const double lo = lib.cell_lo[ag], hi = lib.cell_hi[ag];
    // first bin whose upper edge exceeds lo
    int i = 0;
    {
      int l = 0, h = n_sfh;   // search over edges[1..n_sfh]
      while (l < h) {
        int mid = (l + h) >> 1;
        if (edges[mid + 1] > lo) h = mid; else l = mid + 1;
      }
      i = l;
    }
    for (; i < n_sfh && edges[i] < hi; ++i) {
      const double Ti = edges[i], Tj = edges[i + 1];
      const double ov = fmin(hi, Tj) - fmax(lo, Ti);
      if (ov <= 0.0) continue;
      const double w = mass[i] * ov / (Tj - Ti);
      const int j = zj[i];
      const double t = zt[i];
      for (int q = 0; q < (nf > 1 ? 2 : 1); ++q) {
        const int ia = nf > 1 ? ja + q : 0;
        const double fa = nf > 1 ? (q == 0 ? 1.0 - ta : ta) : 1.0;
        const int base = ia * nz;
        if (nz > 1) {
          wacc[kpos_of(lib, ia, j, ag)] += fa * (1.0 - t) * w;
          wacc[kpos_of(lib, ia, j + 1, ag)] += fa * t * w;
        } else {
          wacc[kpos_of(lib, ia, 0, ag)] += fa * w;
        }
      }
    }
  }
  __syncthreads();

  // ---- nebular lines (App. C): L_l = sum_a 10^Lhat_l(a) sum_{alpha,m} W Q
  const int slot = a.point_obs ? a.point_obs[b] : 0;
  const int kind = a.obs_table[slot].kind;
  const int ny = lib.n_young;
  if (lib.n_line > 0) {
    for (int ag = tid; ag < ny; ag += 256) {
      double s = 0.0;
      for (int ia = 0; ia < nf; ++ia)
        for (int m = 0; m < nz; ++m)
          s += wacc[kpos_of(lib, ia, m, ag)] * lib.Q[(ia * nz + m) * ny + ag];
      wq[ag] = s;
    }
    __syncthreads();
    int jg = 0, ju = 0;
    double tg = 0.0, tu = 0.0;
    bool in;
    grid_split_dev(lib.zg, lib.n_zg, s_th[TH_GAS_LOGZ], jg, tg, in);
    grid_split_dev(lib.un, lib.n_u, s_th[TH_GAS_LOGU], ju, tu, in);
    const int nu = lib.n_u;
    double *lt = wq + ny;   // [n_line * n_young] per (line, age) luminosity terms
    for (int q = tid; q < lib.n_line * ny; q += 256) {
      const int l = q / ny, ag = q - l * ny;
      const size_t slab = (size_t)lib.n_line * ny;
      const double *tb = lib.line_table + q;
      const double lh = (1.0 - tg) * (1.0 - tu) * tb[(jg * nu + ju) * slab] +
                        (1.0 - tg) * tu * tb[(jg * nu + ju + 1) * slab] +
                        tg * (1.0 - tu) * tb[((jg + 1) * nu + ju) * slab] + tg * tu * tb[((jg + 1) * nu + ju + 1) * slab];
      lt[q] = exp10(lh) * wq[ag];
    }
    __syncthreads();
    for (int l = tid; l < lib.n_line; l += 256) {
      double Ll = 0.0;
      for (int ag = 0; ag < ny; ++ag) Ll += lt[l * ny + ag];
      if (kind == 0) wacc[a.line_k0 + l] = Ll / kLsun;        // photometry: lines on the model grid
      else a.Lline[(size_t)r * lib.n_line + l] = Ll;           // spectra: lines on the detector pixels
    }
    __syncthreads();
  }

  // ---- write the row in the contraction's format and its K-tile occupancy bits
  double wscale = 1.0;
  if (MODE == W_F64 || MODE == W_F32) {
    for (int k = tid; k < K_pad; k += 256) {
      if (MODE == W_F64) ((double *)a.W)[(size_t)r * K_pad + k] = wacc[k];
      else ((float *)a.W)[(size_t)r * K_pad + k] = (float)wacc[k];
    }
  } else {
    // W'_k = W_k 2^{e_k}; row scale 2^{e_b} puts max |W'| in [2^14, 2^15)
    double mx = 0.0;
    for (int k = tid; k < K_pad; k += 256) mx = fmax(mx, fabs(ldexp(wacc[k], lib.kexp[k])));
    mx = block_max<256>(mx, red);
    int eb = 0;
    if (mx > 0.0) eb = ilogb(mx) - 14;
    wscale = ldexp(1.0, eb);
    uint16_t *hi = (uint16_t *)a.W, *lo = (uint16_t *)a.Wlo;
    for (int k = tid; k < K_pad; k += 256) {
      const double x = ldexp(wacc[k], lib.kexp[k] - eb);
      uint16_t h, l;
      if (MODE == W_BF16) {
        h = bf16_rne((float)x);
        l = bf16_rne((float)(x - (double)bf16_to_f(h)));
      } else {
        h = f16_rne((float)x);
        l = f16_rne((float)(x - (double)f16_to_f(h)));
      }
      hi[(size_t)r * K_pad + k] = h;
      lo[(size_t)r * K_pad + k] = l;
      wacc[k] = (h != 0 || l != 0) ? 1.0 : 0.0;   // reuse the LDS row for the occupancy test
    }
  }
  __syncthreads();
  {
    uint32_t *tbits = (uint32_t *)red;   // reuse: one word per 32 K tiles
    for (int w = tid; w < a.mask_words; w += 256) tbits[w] = 0u;
    __syncthreads();
    const int n_kt = K_pad / kKTile;
    for (int t = tid; t < n_kt; t += 256) {
      bool on = false;
      for (int k = t * kKTile; k < (t + 1) * kKTile; ++k) on |= (wacc[k] != 0.0);
      if (on) atomicOr(&tbits[t >> 5], 1u << (t & 31));
    }
    __syncthreads();
    for (int w = tid; w < a.mask_words; w += 256) a.rowmask[(size_t)r * a.mask_words + w] = tbits[w];
  }

  if (tid == 0) {
    PointRow pr;
    pr.z = z;
    pr.t_univ = t_univ;
    pr.dl = dl;
    pr.dc = dc;
    pr.mass10 = exp10(s_th[TH_LOGMASS]);
    pr.scale_fnu = pr.mass10 * (1.0 + z) / (4.0 * kPi * dl * dl) * kLsun * kAng_cm / kC_cms;
    pr.wscale = wscale;
    pr.tau_bc = s_th[TH_TAU_BC];
    pr.alpha_bc = s_th[TH_ALPHA_BC];
    pr.tau_diff = s_th[TH_TAU_DIFF];
    pr.delta = s_th[TH_DELTA];
    pr.b = b;
    pr.obs = slot;
    pr.kind = kind;
    pr.pad = 0;
    a.rows[r] = pr;
  }
}

// ---------------------------------------------------------------------------------
// Active K-tile list per M tile (OR of the row masks).  Tiles of kKTile * tf columns.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tiles(const uint32_t *__restrict__ rowmask, int mask_words, int MT,
                                               int n_tiles32, int young_tiles32, int tf, int *__restrict__ tiles,
                                               int *__restrict__ n_young, int *__restrict__ n_act,
                                               unsigned long long *__restrict__ counter) {
  __shared__ uint32_t acc[64];
  __shared__ int cnt[256], cy[256];
  const int mt = blockIdx.x, tid = threadIdx.x;
  if (tid < 64) acc[tid] = 0u;
  __syncthreads();
  for (int idx = tid; idx < MT * mask_words; idx += 256) {
    const int r = idx / mask_words, w = idx - r * mask_words;
    const uint32_t v = rowmask[(size_t)(mt * MT + r) * mask_words + w];
    if (v) atomicOr(&acc[w], v);
  }
  __syncthreads();
  const int n_tiles = (n_tiles32 + tf - 1) / tf;
  const int y_tiles = young_tiles32 / tf;
  const int chunk = (n_tiles + 255) / 256;
  const int t0 = min(tid * chunk, n_tiles), t1 = min(t0 + chunk, n_tiles);
  auto on_tile = [&](int t) {
    bool on = false;
    for (int q = 0; q < tf; ++q) {
      const int t32 = t * tf + q;
      if (t32 < n_tiles32) on |= (acc[t32 >> 5] >> (t32 & 31)) & 1u;
    }
    return on;
  };
  int c = 0, y = 0;
  for (int t = t0; t < t1; ++t)
    if (on_tile(t)) {
      ++c;
      y += t < y_tiles;
    }
  cnt[tid] = c;
  cy[tid] = y;
  __syncthreads();
  // inclusive scan of cnt (Hillis-Steele), sum of cy
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (tid < s2) cy[tid] += cy[tid + s2];
    __syncthreads();
  }
  int pos = cnt[tid] - c;
  for (int t = t0; t < t1; ++t)
    if (on_tile(t)) tiles[mt * n_tiles + pos++] = t;
  if (tid == 0) {
    n_act[mt] = cnt[255];
    n_young[mt] = cy[0];
    if (counter) atomicAdd(counter, (unsigned long long)cnt[255]);
  }
}

// ---------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------
size_t prep_smem_bytes(const DevLib &lib) {
  return sizeof(double) * ((size_t)lib.K_pad + lib.n_sfh + 1 + lib.n_sfh + 256 + lib.n_young +
                           (size_t)lib.n_line * lib.n_young + 8) +
         sizeof(int) * ((size_t)lib.n_sfh + 2);
}

hipError_t launch_sort(const DevLib &lib, const double *theta, int P, int B, double *keys, int *perm, hipStream_t s) {
  hipLaunchKernelGGL(k_keys, dim3((B + 255) / 256), dim3(256), 0, s, lib, theta, P, B, keys);
  hipLaunchKernelGGL(k_sort, dim3(B), dim3(256), 0, s, keys, B, perm);
  return hipGetLastError();
}

hipError_t launch_prep(const DevLib &lib, const PrepLaunch &pl, hipStream_t s) {
  PrepArgs a;
  a.theta = pl.theta;
  a.P = pl.P;
  a.B = pl.B;
  a.B_pad = pl.B_pad;
  a.perm = pl.perm;
  a.obs_table = pl.obs_table;
  a.point_obs = pl.point_obs;
  a.W = pl.W;
  a.Wlo = pl.Wlo;
  a.rowmask = pl.rowmask;
  a.mask_words = pl.mask_words;
  a.rows = pl.rows;
  a.Lline = pl.Lline;
  a.kpos = pl.kpos;
  a.line_k0 = pl.line_k0;
  const size_t sm = prep_smem_bytes(lib);
  if (sm > 160 * 1024) return hipErrorInvalidValue;
  static size_t attr_set[4] = {0, 0, 0, 0};
  const void *fn[4] = {(const void *)k_prep<W_F64>, (const void *)k_prep<W_F32>, (const void *)k_prep<W_BF16>,
                       (const void *)k_prep<W_F16>};
  const int md = pl.mode & 3;
  if (sm > 48 * 1024 && sm > attr_set[md]) {
    hipError_t e = hipFuncSetAttribute(fn[md], hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    attr_set[md] = sm;
  }
  const dim3 g(pl.B_pad), blk(256);
  switch (pl.mode) {
    case W_F64: hipLaunchKernelGGL(k_prep<W_F64>, g, blk, sm, s, lib, a); break;
    case W_F32: hipLaunchKernelGGL(k_prep<W_F32>, g, blk, sm, s, lib, a); break;
    case W_BF16: hipLaunchKernelGGL(k_prep<W_BF16>, g, blk, sm, s, lib, a); break;
    default: hipLaunchKernelGGL(k_prep<W_F16>, g, blk, sm, s, lib, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_tiles(const uint32_t *rowmask, int mask_words, int B_pad, int MT, int n_tiles32, int young_tiles32,
                        int tf, int *tiles, int *n_young, int *n_act, unsigned long long *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_tiles, dim3(B_pad / MT), dim3(256), 0, s, rowmask, mask_words, MT, n_tiles32, young_tiles32,
                     tf, tiles, n_young, n_act, counter);
  return hipGetLastError();
}

}  // namespace sps
