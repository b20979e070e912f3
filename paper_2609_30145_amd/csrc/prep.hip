// Per-point preparation: batch ordering, cosmology, SFH x ZH -> SSP weights, nebular
// line luminosities and the K-tile occupancy of the contraction.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace sps {


// ---------------------------------------------------------------------------------
// Batch ordering.  Rows that share a redshift (time-varying enrichment) or a
// metallicity/alpha bracket (constant metallicity) are grouped so that whole
// K tiles of the weight matrix are zero for an M tile and can be skipped.
// ---------------------------------------------------------------------------------
// The key of a row: its redshift (time-varying enrichment), else the metallicity and
// alpha brackets, then the redshift.
// A redshift that is not a number sorts last (+inf), so that ties are broken by the batch
// index and every row still takes a distinct rank; its own outputs come out non-finite.
__device__ double sort_key(const DevLib &lib, const double *th) {
  double z = th[TH_ZRED];
  if (z != z) z = HUGE_VAL;
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

// Rank of every point in the key order, ties by batch index: rank[b] = #{j : key_j < key_b
// or (key_j == key_b and j < b)}.  A workgroup takes 64 points (one per lane); the batch's
// keys stream through LDS 4096 at a time and each wave compares its lanes' keys against its
// quarter of every chunk (the keys are read once per 64 points, not once per point).  For
// large batches only (kRankKernelMinB): below that the weight builder ranks its own point,
// which saves a launch.
__global__ void __launch_bounds__(256) k_rank(const double *__restrict__ keys, int B, int *__restrict__ ranks) {
  constexpr int CH = 4096;   // keys per chunk in LDS (32 KB), sixteen loads per thread in flight
  __shared__ double s_k[CH];
  __shared__ int s_c[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int b = blockIdx.x * 64 + lane;
  const double my = keys[min(b, B - 1)];
  int c = 0;
  for (int j0 = 0; j0 < B; j0 += CH) {
    double v[CH / 256];
#pragma unroll
    for (int q = 0; q < CH / 256; ++q) v[q] = keys[min(j0 + tid + 256 * q, B - 1)];
#pragma unroll
    for (int q = 0; q < CH / 256; ++q) s_k[tid + 256 * q] = v[q];
    __syncthreads();
    // wave wv compares its lanes' keys with the chunk's keys wv, wv + 4, wv + 8, ...
    const int n = min(CH, B - j0);
    const int full = n & ~63;
    for (int u0 = wv * 16; u0 < full; u0 += 64) {
      double kk[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) kk[w] = s_k[u0 + w];
#pragma unroll
      for (int w = 0; w < 16; ++w) {
        const int j = j0 + u0 + w;
        c += (kk[w] < my) || (kk[w] == my && j < b);
      }
    }
    for (int u = full + wv; u < n; u += 4) {
      const double k = s_k[u];
      const int j = j0 + u;
      c += (k < my) || (k == my && j < b);
    }
    __syncthreads();
  }
  s_c[wv][lane] = c;
  __syncthreads();
  if (wv == 0 && b < B) ranks[b] = (s_c[0][lane] + s_c[1][lane]) + (s_c[2][lane] + s_c[3][lane]);
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

// Position of weight (row r, K entry k) in the 16-bit planes, which the contraction
// reads straight into MFMA registers: blocks of 32 rows x 64 K entries (4 KB), inside a
// block chunk-major ([8-entry chunk][row][8]), so one wave load of a chunk for its 32
// rows is a single contiguous 512-byte run.
__device__ __forceinline__ size_t w16_pos(int r, int k, int n_kt64) {
  return ((size_t)(r >> 5) * n_kt64 + (k >> 6)) * 2048 + (size_t)((k >> 3) & 7) * 256 + (r & 31) * 8 + (k & 7);
}

// Output mode of the weight row.
enum WMode { W_F64 = 0, W_F32 = 1, W_BF16 = 2, W_F16 = 3 };

struct PrepArgs {
  const double *theta;
  int P, B, B_pad;
  const double *keys;       // [B] batch-ordering keys (k_keys), or NULL: formed here (B <= kSelfKeyMaxB)
  const int *ranks;         // [B] each point's row in the key order (k_rank), or NULL: ranked here
  const DevObs *obs_table;
  const int *point_obs;     // [B] observation slot per point, NULL = slot 0
  void *W;                  // F64/F32: [B_pad][K_pad]; 16-bit: hi plane
  void *Wlo;                // 16-bit residual plane
  uint32_t *rowmask;        // [B_pad][mask_words]
  int mask_words;
  PointRow *rows;           // [B_pad]
  double *Lline;            // [B_pad][n_line] (spectra: line luminosities, erg/s per Msun)
  double *WQ;               // [B_pad][neb_a1 - neb_a0] sum_{alpha,m} W Q per nebular age / kWqScale, or NULL
  const int *kpos;          // [n_afe][n_z][n_age] -> K position
  int line_k0;              // K position of line 0 (photometric path)
};

// bracketing node j and fraction t of x on a short grid held in LDS, clamped; the
// same (j, t) as grid_split_dev by bisection
__device__ __forceinline__ void split_lds(const double *nodes, int n, double x, int &j, double &t) {
  const double xc = fmin(fmax(x, nodes[0]), nodes[n - 1]);
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (nodes[mid] <= xc) lo = mid; else hi = mid;
  }
  j = lo;
  t = (xc - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// LDS layout of k_prep, in 8-byte words (the weight row and the line terms are
// FP64 for the FP64 path and FP32 otherwise).  The node tables (logz .. Q) are one
// contiguous run in the order of DevLib::prep_tab, so that they arrive in one copy.
struct PrepSmem {
  int th, logz, afe, clo, chi, zg, un, Q, ages, edges, mr, zt, zj, wq, ke, wacc, lt, lr, pc, pidx, total;
  __host__ __device__ PrepSmem(const DevLib &lib, int mode) {
    const bool f64 = mode == 0, w16 = mode >= 2;
    const int acc = f64 ? 8 : 4;
    int o = 0;
    th = o;    o += lib.P;
    logz = o;  o += lib.n_z;
    afe = o;   o += lib.n_afe;
    clo = o;   o += lib.n_age;
    chi = o;   o += lib.n_age;
    zg = o;    o += lib.n_zg;
    un = o;    o += lib.n_u;
    Q = o;
    ages = Q + (lib.has_neb ? lib.n_afe * lib.n_z * lib.n_young : 0);   // linear SFH scheme only
    o = logz + prep_tab_len(lib);                          // Q, the ages and the block's padding
    edges = o; o += lib.n_sfh + 1;
    mr = o;    o += lib.n_sfh;                             // bin mass per unit time
    zt = o;    o += lib.n_sfh;
    zj = o;    o += (lib.n_sfh + 1) / 2;                  // int
    wq = o;    o += lib.has_neb ? lib.n_young : 0;
    ke = o;    o += w16 ? lib.K_pad / 4 : 0;              // int16 row exponents
    wacc = o;  o += (lib.K_pad * acc + 7) / 8;
    lt = o;    o += (lib.n_line * lib.n_young * acc + 7) / 8;
    lr = o;    o += lib.sfh_scheme ? lib.n_age : 0;       // ln(t_a / t_{a-1}) (linear scheme)
    // linear scheme: the tent masses of the (bin, node) pairs whose intervals overlap.  A
    // tent spans two of the n_age + 1 cells between nodes, and a bin partition and a cell
    // partition of one line overlap in at most n_sfh + n_age + 1 pairs, so 2 (n_sfh +
    // n_age + 1) pairs, plus two per bin of zero width (one point inside at most two tents)
    pc = o;    o += lib.sfh_scheme ? 4 * lib.n_sfh + 2 * lib.n_age + 2 : 0;
    pidx = o;  o += lib.sfh_scheme ? lib.n_sfh + 1 : 0;     // int: each bin's first node, pair offsets
    total = o;
  }
};

// Linear SFH scheme (App. B, eq. tent_integral): the mass an SFH bin [T0, T1] with SFR
// linear from p0 to p1 gives SSP age node ag: the integral of the SFR against the node's
// tent (linear in ln t between neighbouring nodes; the whole interval below the first node
// and above the last), the pieces added in the order lower end, lower half, upper half,
// upper end.  Each piece [u, v] is written about its own start u, the SFR as
// psi(u) + beta (t - u) and ln t as ln u + ln(1 + x), x = (t - u)/u, so that no large terms
// cancel: with A = int_0^X ln(1+x) dx and B = int_0^X x ln(1+x) dx (X = (v - u)/u, closed
// forms, or Taylor series below X = 0.05), int psi = (v - u)(psi(u) + beta (v - u)/2) and
// I = int psi ln(t/u) = u (psi(u) A + beta u B); the lower half takes ln(u/t_{ag-1}) int psi
// + I and the upper half ln(t_{ag+1}/u) int psi - I, each over ln(t_{ag+1}/t_ag).
// Taylor coefficients of A / X^2 ((-1)^k / (k (k - 1)), k = 2 .. 15) and of B / X^3
// ((-1)^(n+1) / (n (n + 2)), n = 1 .. 14), rounded once at compile time
struct LogMomentSeries {
  double a[14], b[14];
  constexpr LogMomentSeries() : a(), b() {
    for (int k = 2; k <= 15; ++k) a[k - 2] = ((k & 1) ? -1.0 : 1.0) / (double)(k * (k - 1));
    for (int n = 1; n <= 14; ++n) b[n - 1] = ((n & 1) ? 1.0 : -1.0) / (double)(n * (n + 2));
  }
};
__device__ constexpr LogMomentSeries kLogMomentSeries{};

__device__ __forceinline__ void log_moments(double X, double &A, double &B) {
  if (X < 0.05) {
    // Horner from the highest power
    double a = kLogMomentSeries.a[13], b = kLogMomentSeries.b[13];
#pragma unroll
    for (int k = 12; k >= 0; --k) {
      a = __fma_rn(a, X, kLogMomentSeries.a[k]);
      b = __fma_rn(b, X, kLogMomentSeries.b[k]);
    }
    A = a * X * X;
    B = b * X * X * X;
  } else {
    const double lp = log1p(X);
    A = (1.0 + X) * lp - X;
    B = 0.5 * (X * X - 1.0) * lp - 0.25 * X * X + 0.5 * X;
  }
}

// lr[a] = ln(t_a / t_{a-1}) (a >= 1), formed once per point; the logarithms of a piece's
// end over a node are taken only where the end is not the node itself.
__device__ double tent_mass(const double *ages, const double *lr, int na, int ag, double T0, double T1, double p0,
                            double p1) {
  const double beta = (p1 - p0) / (T1 - T0);
  auto at = [&](double x) { return p0 + beta * (x - T0); };
  auto piece = [&](double u, double v, double &i0, double &I) {
    double A, B;
    log_moments((v - u) / u, A, B);
    const double pu = at(u);
    i0 = (v - u) * (pu + 0.5 * beta * (v - u));
    I = u * (pu * A + beta * u * B);
  };
  double c = 0.0;
  if (ag == 0) {
    const double u = T0, v = fmin(T1, ages[0]);
    if (v > u) c += (v - u) * (at(u) + 0.5 * beta * (v - u));
  }
  if (ag > 0) {   // weight ln(t / t_{ag-1}) / ln(t_ag / t_{ag-1}) on [t_{ag-1}, t_ag]
    const double u = fmax(T0, ages[ag - 1]), v = fmin(T1, ages[ag]);
    if (v > u) {
      double i0, I;
      piece(u, v, i0, I);
      c += ((u == ages[ag - 1] ? 0.0 : log(u / ages[ag - 1])) * i0 + I) / lr[ag];
    }
  }
  if (ag + 1 < na) {   // weight ln(t_{ag+1} / t) / ln(t_{ag+1} / t_ag) on [t_ag, t_{ag+1}]
    const double u = fmax(T0, ages[ag]), v = fmin(T1, ages[ag + 1]);
    if (v > u) {
      double i0, I;
      piece(u, v, i0, I);
      c += ((u == ages[ag] ? lr[ag + 1] : log(ages[ag + 1] / u)) * i0 - I) / lr[ag + 1];
    }
  }
  if (ag == na - 1) {
    const double u = fmax(T0, ages[na - 1]), v = T1;
    if (v > u) c += (v - u) * (at(u) + 0.5 * beta * (v - u));
  }
  return c;
}

// One workgroup (4 waves) per sorted row:
//   A1  every global load of the phase in flight together: theta, the node-table block,
//       the 16-bit row exponents, the first batch keys, the quadrature nodes; then the
//       point's rank among the batch keys, the Gauss-Legendre partial sums of D_C
//       (waves 0-2) and t_univ with the SFH bin edges (wave 3)
//   A2  the bin metallicities and their bracketing nodes, the bin mass per unit time;
//       the interpolated line terms 10^Lhat (they depend on the gas parameters only)
//   B   step-scheme overlap weights, one thread per SSP age (single writer per slot)
//   C   photon-weighted young mass per age, then the line luminosities
//   D   the row in the contraction's format with its K-tile occupancy bits, eight
//       consecutive K entries per thread; the per-point row (redshift, distances, scales).
// LINEAR: the SFH scheme (lib.sfh_scheme), a template argument so that the step scheme's
// kernel does not carry the tent integrals' registers
template <int MODE, bool LINEAR>
__global__ void __launch_bounds__(256) k_prep(DevLib lib, PrepArgs a) {
  using Acc = typename std::conditional<MODE == W_F64, double, float>::type;
  constexpr bool W16 = MODE == W_BF16 || MODE == W_F16;
  extern __shared__ double smem[];
  const PrepSmem L(lib, MODE);
  const int K_pad = lib.K_pad, na = lib.n_age, nz = lib.n_z, nf = lib.n_afe, ny = lib.n_young;
  const int n_sfh = lib.n_sfh, nl = lib.n_line;
  double *s_th = smem + L.th, *s_logz = smem + L.logz, *s_afe = smem + L.afe;
  double *s_clo = smem + L.clo, *s_chi = smem + L.chi, *s_zg = smem + L.zg, *s_un = smem + L.un;
  double *s_Q = smem + L.Q, *s_edges = smem + L.edges, *s_mr = smem + L.mr, *s_zt = smem + L.zt;
  const double *s_ages = smem + L.ages;
  double *s_lr = smem + L.lr;
  double *s_pc = smem + L.pc;
  int *s_plo = (int *)(smem + L.pidx), *s_poff = s_plo + n_sfh;
  double *s_wq = smem + L.wq;
  int *s_zj = (int *)(smem + L.zj);
  const int16_t *s_ke = (const int16_t *)(smem + L.ke);
  Acc *wacc = (Acc *)(smem + L.wacc);
  Acc *s_lt = (Acc *)(smem + L.lt);
  __shared__ double s_part[4];
  __shared__ double s_tu, s_m10;
  __shared__ uint32_t s_bits[64];
  __shared__ int s_rank[4];

  // workgroup b takes point b (caller's order); its row r is the point's rank in the
  // key order (ties by index).  Workgroups past B clear the padding rows.
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int b = blockIdx.x < a.B ? blockIdx.x : -1;
  if (b < 0) {   // padding row: zero weights
    const int r = blockIdx.x;
    const size_t rowoff = (size_t)r * K_pad;
    for (int k = tid; k < K_pad; k += 256) {
      if (MODE == W_F64) ((double *)a.W)[rowoff + k] = 0.0;
      else if (MODE == W_F32) ((float *)a.W)[rowoff + k] = 0.f;
      else {
        ((uint16_t *)a.W)[w16_pos(r, k, K_pad >> 6)] = 0;
        ((uint16_t *)a.Wlo)[w16_pos(r, k, K_pad >> 6)] = 0;
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

  // ---- A1.  Loads are issued from clamped indices, unconditionally, so that all of them
  // are in flight before the first use; sizes beyond the unrolled counts take the loops
  // that follow each store.
  constexpr int UT = 2, UB = 4, UK = 4, UQ = 4;
  const double *th = a.theta + (size_t)b * a.P;
  const double z = th[TH_ZRED];
  const int slot = a.point_obs ? a.point_obs[b] : 0;
  const int n_gl = lib.n_gl, gi = min(tid, n_gl - 1);
  const double gu = lib.gl_u[gi], gw = lib.gl_w[gi];
  const int P = a.P, nt2 = prep_tab_len(lib) >> 1, nk8 = K_pad >> 3;
  const double2 *tab2 = (const double2 *)lib.prep_tab;
  const uint4 *ke4 = (const uint4 *)lib.kexp16;
  double vt[UT];
  double2 vb[UB];
  uint4 vk[UK];
#pragma unroll
  for (int u = 0; u < UT; ++u) vt[u] = th[min(tid + 256 * u, P - 1)];
#pragma unroll
  for (int u = 0; u < UB; ++u) vb[u] = tab2[min(tid + 256 * u, nt2 - 1)];
  if (W16) {
#pragma unroll
    for (int u = 0; u < UK; ++u) vk[u] = ke4[min(tid + 256 * u, nk8 - 1)];
  }
  double kq[UQ], my = 0.0;
  if (!a.ranks && a.keys) {   // small batches rank themselves (no k_rank launch)
#pragma unroll
    for (int u = 0; u < UQ; ++u) kq[u] = a.keys[min(tid + 256 * u, a.B - 1)];
    my = a.keys[b];
  } else if (!a.ranks) {      // the smallest ones also form the keys here (no k_keys launch)
#pragma unroll
    for (int u = 0; u < UQ; ++u) {
      const int j = tid + 256 * u;
      kq[u] = j < a.B ? sort_key(lib, a.theta + (size_t)j * a.P) : 0.0;
    }
    my = sort_key(lib, th);
  }

  // cosmology (Sec. 2.6): D_C by composite Gauss-Legendre in u = (1+z')^-1/2, where
  // the integrand 2 / sqrt(Om + OL u^6) is smooth (waves 0-2); t_univ in closed form
  // and the SFH edges rescaled to it (App. B): T_0 = 0, T_1 = T1, T_n = t_univ,
  // log-uniform in between (wave 3)
  const double Om = lib.Om, OL = 1.0 - lib.Om;
  const double u0 = 1.0 / sqrt(1.0 + z);
  if (wv < 3) {
    double part = 0.0;
    if (tid < n_gl) {
      const double u = u0 + (1.0 - u0) * gu;
      const double u2 = u * u;
      part = gw * 2.0 / sqrt(Om + OL * u2 * u2 * u2);
    }
    for (int i = tid + 192; i < n_gl; i += 192) {
      const double u = u0 + (1.0 - u0) * lib.gl_u[i];
      const double u2 = u * u;
      part += lib.gl_w[i] * 2.0 / sqrt(Om + OL * u2 * u2 * u2);
    }
    part = wave_sum(part);
    if (lane == 0) s_part[wv] = part;
    // the mass scale 10^logmass, off the critical path (wave 2 has no quadrature nodes
    // while n_gl <= 128)
    if (wv == 2 && lane == 0) s_m10 = exp10(th[TH_LOGMASS]);
  } else {
    // (1+z)^{-3/2} by a square root and asinh(x) = ln(x + sqrt(x^2 + 1)) for x > 0: a
    // shorter chain of double-precision operations than the library pow and asinh
    const double tH_yr = kMpc_km / lib.H0 / kYr_s;
    const double opz = 1.0 + z;
    const double x = sqrt(OL / Om) / (opz * sqrt(opz));
    const double tu = tH_yr * 2.0 / (3.0 * sqrt(OL)) * log(x + sqrt(x * x + 1.0));
    const double lnR = log(tu / lib.T1);
    for (int i = lane; i <= n_sfh; i += 64) {
      double T;
      if (i == 0) T = 0.0;
      else if (i == 1) T = lib.T1;
      else if (i == n_sfh) T = tu;
      else T = lib.T1 * exp(lnR * (double)(i - 1) / (double)(n_sfh - 1));
      s_edges[i] = T;
    }
    if (lane == 0) {
      s_tu = tu;
      s_part[3] = 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < UT; ++u)
    if (tid + 256 * u < P) s_th[tid + 256 * u] = vt[u];
  for (int c = tid + 256 * UT; c < P; c += 256) s_th[c] = th[c];
#pragma unroll
  for (int u = 0; u < UB; ++u) {
    const int i = tid + 256 * u;
    if (i < nt2) {
      s_logz[2 * i] = vb[u].x;
      s_logz[2 * i + 1] = vb[u].y;
    }
  }
  for (int i = tid + 256 * UB; i < nt2; i += 256) {
    const double2 v = tab2[i];
    s_logz[2 * i] = v.x;
    s_logz[2 * i + 1] = v.y;
  }
  if (W16) {
    uint2 *ke2 = (uint2 *)(smem + L.ke);
#pragma unroll
    for (int u = 0; u < UK; ++u) {
      const int i = tid + 256 * u;
      if (i < nk8) {
        ke2[2 * i] = make_uint2(vk[u].x, vk[u].y);
        ke2[2 * i + 1] = make_uint2(vk[u].z, vk[u].w);
      }
    }
    for (int i = tid + 256 * UK; i < nk8; i += 256) {
      const uint4 v = ke4[i];
      ke2[2 * i] = make_uint2(v.x, v.y);
      ke2[2 * i + 1] = make_uint2(v.z, v.w);
    }
  }
  for (int k = tid; k < K_pad; k += 256) wacc[k] = (Acc)0;
  if (tid < 64) s_bits[tid] = 0u;
  int r;   // the point's row: its rank in the key order, ties by index
  if (a.ranks) {
    r = a.ranks[b];
    __syncthreads();
  } else {
    int c = 0;
#pragma unroll
    for (int u = 0; u < UQ; ++u) {
      const int j = tid + 256 * u;
      c += j < a.B && ((kq[u] < my) || (kq[u] == my && j < b));
    }
    for (int j0 = tid + 256 * UQ; j0 < a.B; j0 += 256 * 4) {   // four key loads per thread in flight
      double kk[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) kk[u] = a.keys[min(j0 + 256 * u, a.B - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + 256 * u;
        c += j < a.B && ((kk[u] < my) || (kk[u] == my && j < b));
      }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) s_rank[wv] = c;
    __syncthreads();
    r = (s_rank[0] + s_rank[1]) + (s_rank[2] + s_rank[3]);
  }
  const size_t rowoff = (size_t)r * K_pad;
  const double dc = kC_kms / lib.H0 * (1.0 - u0) * ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])) * kMpc_cm;
  // the point's observation kind and filter span, requested here and first used in
  // phase C and at the end
  const DevObs *obp = a.obs_table + slot;
  const int kind = obp->kind;
  const double fw_min = obp->fwln_min, fw_max = obp->fwln_max;
  const double px_lo = obp->lnpix_lo, px_hi = obp->lnpix_hi, ks_max = obp->ksig_max;
  const double vd_lo = obp->vd_lnlo, vd_hi = obp->vd_lnhi, vd_dl = obp->vd_dlnl;
  const int vd_M = obp->vd_M, vd_n = obp->vd_nfft;

  if (LINEAR) {   // the age nodes' log ratios for the tent integrals
    for (int ag = 1 + tid; ag < na; ag += 256) s_lr[ag] = log(s_ages[ag] / s_ages[ag - 1]);
    __syncthreads();
  }

  // ---- A2: bin metallicity from the enrichment history (Sec. 2.2.2): nodes and bin
  // centres are both log-uniform from T1 to t_univ, so the interpolation weight in ln T
  // is fixed in the normalised coordinate (bin i >= 1 at (i - 1/2)/(n_sfh - 1), node k
  // at k/(n_zh - 1)); the first bin (centre T1/2) takes node 0
  {
    const double *zh = s_th + TH_NSCALAR + n_sfh;
    for (int i = tid; i < n_sfh; i += 256) {
      double zeta;
      if (lib.n_zh == 0) {
        zeta = s_th[TH_LOGZSOL];
      } else if (i == 0) {
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
      if (nz > 1) split_lds(s_logz, nz, zeta, j, t);
      s_zj[i] = j;
      s_zt[i] = t;
      if (!LINEAR) {
        s_mr[i] = s_th[TH_NSCALAR + i] / (s_edges[i + 1] - s_edges[i]);
      } else {
        // linear scheme: the nodes whose tents [t_{ag-1}, t_{ag+1}] meet the bin, in
        // increasing order: from the first whose tent ends above T0 (bisection) while the
        // tent starts below T1; their count, and the bin's trapezoid mass (p_i + p_{i+1})
        // (T_{i+1} - T_i) / 2 (the last SFR repeated), which the tent masses are rescaled to
        const double p0 = s_th[TH_NSCALAR + i], p1 = s_th[TH_NSCALAR + min(i + 1, n_sfh - 1)];
        const double T0 = s_edges[i], T1 = s_edges[i + 1];
        int ag = 0;
        {
          int l = 0, h = na - 1;
          while (l < h) {
            const int mid = (l + h) >> 1;
            if (s_ages[mid + 1] > T0) h = mid; else l = mid + 1;
          }
          ag = l;
        }
        s_plo[i] = ag;
        int cnt = 0;
        for (; ag < na && (ag == 0 ? 0.0 : s_ages[ag - 1]) < T1; ++ag) ++cnt;
        s_poff[i + 1] = cnt;
        s_mr[i] = 0.5 * (p0 + p1) * (T1 - T0);
      }
    }
  }
  if (nl > 0) {
    // 10^Lhat_l(a): bilinear in (log Z_gas, log U) of the tabulated log values (App. C);
    // entry q = l * n_young + a, consecutive threads on consecutive entries
    int jg = 0, ju = 0;
    double tg = 0.0, tu = 0.0;
    split_lds(s_zg, lib.n_zg, s_th[TH_GAS_LOGZ], jg, tg);
    split_lds(s_un, lib.n_u, s_th[TH_GAS_LOGU], ju, tu);
    const int nu = lib.n_u;
    const size_t slab = (size_t)nl * ny;
    const size_t o00 = (size_t)(jg * nu + ju) * slab, o01 = (size_t)(jg * nu + ju + 1) * slab;
    const size_t o10 = (size_t)((jg + 1) * nu + ju) * slab, o11 = (size_t)((jg + 1) * nu + ju + 1) * slab;
    const double c00 = (1.0 - tg) * (1.0 - tu), c01 = (1.0 - tg) * tu, c10 = tg * (1.0 - tu), c11 = tg * tu;
    const int nq = nl * ny;
    if (MODE != W_F64 && (nq & 3) == 0) {
      // 16-byte loads: a thread's four consecutive entries of each corner in one request,
      // up to four requests per corner in flight (nq is a multiple of 4, so are the
      // corner offsets, and the table is 16-byte aligned)
      const float4 *tb = (const float4 *)lib.line_table_f;
      const float f00 = (float)c00, f01 = (float)c01, f10 = (float)c10, f11 = (float)c11;
      const int nv = nq >> 2;
      for (int v0 = tid; v0 < nv; v0 += 256 * 4) {
        float4 c[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int v = min(v0 + 256 * u, nv - 1);
          c[u][0] = tb[(o00 >> 2) + v];
          c[u][1] = tb[(o01 >> 2) + v];
          c[u][2] = tb[(o10 >> 2) + v];
          c[u][3] = tb[(o11 >> 2) + v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int v = v0 + 256 * u;
          if (v < nv) {
            const float4 a0 = c[u][0], a1 = c[u][1], a2 = c[u][2], a3 = c[u][3];
            s_lt[4 * v + 0] = (Acc)exp10f(f00 * a0.x + f01 * a1.x + f10 * a2.x + f11 * a3.x);
            s_lt[4 * v + 1] = (Acc)exp10f(f00 * a0.y + f01 * a1.y + f10 * a2.y + f11 * a3.y);
            s_lt[4 * v + 2] = (Acc)exp10f(f00 * a0.z + f01 * a1.z + f10 * a2.z + f11 * a3.z);
            s_lt[4 * v + 3] = (Acc)exp10f(f00 * a0.w + f01 * a1.w + f10 * a2.w + f11 * a3.w);
          }
        }
      }
    } else {
      for (int q0 = tid; q0 < nq; q0 += 256 * 8) {
        if (MODE == W_F64) {
          const double *tb = lib.line_table;
          double lh[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int q = q0 + 256 * u;
            lh[u] = q < nq ? c00 * tb[o00 + q] + c01 * tb[o01 + q] + c10 * tb[o10 + q] + c11 * tb[o11 + q] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int q = q0 + 256 * u;
            if (q < nq) s_lt[q] = (Acc)exp10(lh[u]);
          }
        } else {
          const float *tb = lib.line_table_f;
          const float f00 = (float)c00, f01 = (float)c01, f10 = (float)c10, f11 = (float)c11;
          float lh[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int q = q0 + 256 * u;
            lh[u] = q < nq ? f00 * tb[o00 + q] + f01 * tb[o01 + q] + f10 * tb[o10 + q] + f11 * tb[o11 + q] : 0.f;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int q = q0 + 256 * u;
            if (q < nq) s_lt[q] = (Acc)exp10f(lh[u]);
          }
        }
      }
    }
  }
  __syncthreads();

  if (LINEAR) {
    // the (bin, node) pairs: offsets by an exclusive scan of the bins' counts (wave 0, 64
    // bins at a time), every pair's clipped tent mass once (all threads), then each bin's
    // rescaling factor from its pairs in node order
    if (wv == 0) {
      int carry = 0;
      for (int i0 = 0; i0 < n_sfh; i0 += 64) {
        const int i = i0 + lane;
        int incl = i < n_sfh ? s_poff[i + 1] : 0;
        for (int o = 1; o < 64; o <<= 1) {
          const int v = __shfl_up(incl, o, 64);
          if (lane >= o) incl += v;
        }
        if (i < n_sfh) s_poff[i + 1] = carry + incl;
        carry += __shfl(incl, 63, 64);
      }
      if (lane == 0) s_poff[0] = 0;
    }
    __syncthreads();
    const int n_pairs = s_poff[n_sfh];
    for (int p = tid; p < n_pairs; p += 256) {
      int l = 0, h = n_sfh - 1;   // the pair's bin: the last i with s_poff[i] <= p
      while (l < h) {
        const int mid = (l + h + 1) >> 1;
        if (s_poff[mid] <= p) l = mid; else h = mid - 1;
      }
      const int i = l, ag = s_plo[i] + (p - s_poff[i]);
      const double p0 = s_th[TH_NSCALAR + i], p1 = s_th[TH_NSCALAR + min(i + 1, n_sfh - 1)];
      s_pc[p] = fmax(tent_mass(s_ages, s_lr, na, ag, s_edges[i], s_edges[i + 1], p0, p1), 0.0);
    }
    __syncthreads();
    for (int i = tid; i < n_sfh; i += 256) {
      double sum = 0.0;
      for (int p = s_poff[i]; p < s_poff[i + 1]; ++p) sum += s_pc[p];
      s_mr[i] = sum > 0.0 ? s_mr[i] / sum : 1.0;
    }
    __syncthreads();
  }

  // ---- B: overlap of SFH bin i with the linear-time cell of age ag (App. B)
  int ja = 0;
  double ta = 0.0;
  if (nf > 1) split_lds(s_afe, nf, s_th[TH_AFE], ja, ta);
  for (int ag = tid; ag < na && LINEAR; ag += 256) {
    // linear scheme: every bin under the node's tent, [t_{ag-1}, t_{ag+1}] (from 0 for the
    // first node, to +inf for the last)
    const double lo = ag == 0 ? 0.0 : s_ages[ag - 1], hi = ag == na - 1 ? HUGE_VAL : s_ages[ag + 1];
    int i = 0;
    {
      int l = 0, h = n_sfh;
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (s_edges[mid + 1] > lo) h = mid; else l = mid + 1;
      }
      i = l;
    }
    for (; i < n_sfh && s_edges[i] < hi; ++i) {
      const double c = s_pc[s_poff[i] + (ag - s_plo[i])];   // the pair's clipped tent mass
      if (c == 0.0) continue;
      const double w = c * s_mr[i];
      const int j = s_zj[i];
      const double t = s_zt[i];
      for (int q = 0; q < (nf > 1 ? 2 : 1); ++q) {
        const int ia = nf > 1 ? ja + q : 0;
        const double fa = nf > 1 ? (q == 0 ? 1.0 - ta : ta) : 1.0;
        if (nz > 1) {
          wacc[kpos_of(lib, ia, j, ag)] += (Acc)(fa * (1.0 - t) * w);
          wacc[kpos_of(lib, ia, j + 1, ag)] += (Acc)(fa * t * w);
        } else {
          wacc[kpos_of(lib, ia, 0, ag)] += (Acc)(fa * w);
        }
      }
    }
  }
  for (int ag = tid; ag < na && !LINEAR; ag += 256) {
    const double lo = s_clo[ag], hi = s_chi[ag];
    // first bin whose upper edge exceeds lo
    int i = 0;
    {
      int l = 0, h = n_sfh;
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (s_edges[mid + 1] > lo) h = mid; else l = mid + 1;
      }
      i = l;
    }
    for (; i < n_sfh && s_edges[i] < hi; ++i) {
      const double ov = fmin(hi, s_edges[i + 1]) - fmax(lo, s_edges[i]);
      if (ov <= 0.0) continue;
      const double w = s_mr[i] * ov;
      const int j = s_zj[i];
      const double t = s_zt[i];
      for (int q = 0; q < (nf > 1 ? 2 : 1); ++q) {
        const int ia = nf > 1 ? ja + q : 0;
        const double fa = nf > 1 ? (q == 0 ? 1.0 - ta : ta) : 1.0;
        if (nz > 1) {
          wacc[kpos_of(lib, ia, j, ag)] += (Acc)(fa * (1.0 - t) * w);
          wacc[kpos_of(lib, ia, j + 1, ag)] += (Acc)(fa * t * w);
        } else {
          wacc[kpos_of(lib, ia, 0, ag)] += (Acc)(fa * w);
        }
      }
    }
  }
  __syncthreads();

  // ---- escape geometry (Sec. 2.3.2): f_ob from its theta column, clamped to [0, 1] (a NaN
  //      stays NaN); the young light's birth-cloud transmission bc_p e^{-tau_BC} + bc_q and
  //      the nebular scale neb_s: runaway_bc (1 - f, f, 1 - f), picket (1 - f, 0, 1)
  double fob = 0.0, bc_p = 1.0, bc_q = 0.0, neb_s = 1.0;
  if (lib.escape) {
    const double x = s_th[lib.th_fob];
    fob = x != x ? x : fmin(fmax(x, 0.0), 1.0);
    bc_p = 1.0 - fob;
    if (lib.escape == 1) {
      bc_q = fob;
      neb_s = 1.0 - fob;
    }
    // the ionising rows: W_ma of the nebular ages, times f_ob under runaway_bc (the restored
    // fraction, which bypasses the birth cloud); the picket fence's dust-free pass applies
    // f_ob itself
    const int nion = lib.n_ion;
    const Acc sc = lib.escape == 1 ? (Acc)fob : (Acc)1;
    for (int q = tid; q < nion; q += 256) {
      const int ia = q % nf, m = (q / nf) % nz, ag = lib.neb_a0 + q / (nf * nz);
      wacc[lib.ion_k0 + q] = sc * wacc[kpos_of(lib, ia, m, ag)];
    }
  }

  // ---- C: nebular emission (App. C): the photon-weighted mass sum_{alpha,m} W Q per
  //      nebular age, the line luminosities L_l = sum_a 10^Lhat_l(a) sum_{alpha,m} W Q (the
  //      line table is -1000 outside the nebular ages) and, for the continuum, the per-age
  //      sums themselves
  if (lib.has_neb) {
    // photon-weighted young mass per age: eight lanes per age, each over a strided share
    // of the (alpha, Z) nodes, combined by a fixed butterfly
    const int nm = nf * nz;
    for (int g0 = 0; g0 < ny; g0 += 32) {
      const int ag = g0 + (tid >> 3), c = tid & 7;
      double s = 0.0;
      if (ag < ny)
        for (int q = c; q < nm; q += 8) {
          const int ia = q / nz, m = q - ia * nz;
          s += (double)wacc[kpos_of(lib, ia, m, ag)] * s_Q[q * ny + ag];
        }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      if (ag < ny && c == 0) s_wq[ag] = s;
    }
    __syncthreads();
    if (a.WQ) {
      const int n_nc = lib.neb_a1 - lib.neb_a0;
      for (int q = tid; q < n_nc; q += 256) a.WQ[(size_t)r * n_nc + q] = s_wq[lib.neb_a0 + q] / kWqScale;
    }
  }
  if (nl > 0) {
    // two threads per line (adjacent lanes), each over half of the young ages
    const int half = tid & 1, nyh = (ny + 1) >> 1;
    const int a0 = half ? nyh : 0, a1 = half ? ny : nyh;
    for (int l0 = 0; l0 < nl; l0 += 128) {
      const int l = l0 + (tid >> 1);
      double Ll = 0.0;
      if (l < nl)
        for (int ag = a0; ag < a1; ++ag) Ll += (double)s_lt[l * ny + ag] * s_wq[ag];
      Ll += __shfl_xor(Ll, 1);
      Ll *= neb_s;
      if (l < nl && half == 0) {
        if (kind == 0) wacc[a.line_k0 + l] = (Acc)(Ll / kLsun);   // photometry: lines on the model grid
        else a.Lline[(size_t)r * nl + l] = Ll;                    // spectra: lines on the detector pixels
      }
    }
  }
  __syncthreads();

  // ---- D: the row in the contraction's format and its K-tile occupancy bits.  A thread
  //      takes eight consecutive K entries (one 16-byte run of a 16-bit plane); a wave
  //      covers 512 entries, i.e. 16 tiles of 32, all in one word of the bit mask.
  const int nk8d = K_pad >> 3;
  double wscale = 1.0;
  int eb = 0;
  if (W16) {
    // W'_k = W_k 2^{e_k} (exact in FP32), kept in the LDS row; the row scale 2^{e_b}
    // puts max |W'| in [2^14, 2^15)
    float mx = 0.f;
    for (int c = tid; c < nk8d; c += 256) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * c + e;
        const float x = ldexpf((float)wacc[k], (int)s_ke[k]);
        wacc[k] = (Acc)x;
        mx = fmaxf(mx, fabsf(x));
      }
    }
    double m2 = wave_max((double)mx);
    if (lane == 0) s_part[wv] = m2;   // the D_C partials were read before the A1 barrier
    __syncthreads();
    m2 = fmax(fmax(s_part[0], s_part[1]), fmax(s_part[2], s_part[3]));
    if (m2 > 0.0) eb = ilogb(m2) - 14;
    wscale = ldexp(1.0, eb);
  }
  for (int c = tid; c < nk8d; c += 256) {
    const int k0 = 8 * c;
    bool on = false;
    if (MODE == W_F64) {
      double x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        x[e] = (double)wacc[k0 + e];
        on = on || x[e] != 0.0;
      }
      double2 *dst = (double2 *)((double *)a.W + rowoff + k0);
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = make_double2(x[2 * e], x[2 * e + 1]);
    } else if (MODE == W_F32) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        x[e] = (float)wacc[k0 + e];
        on = on || x[e] != 0.f;
      }
      float4 *dst = (float4 *)((float *)a.W + rowoff + k0);
      dst[0] = make_float4(x[0], x[1], x[2], x[3]);
      dst[1] = make_float4(x[4], x[5], x[6], x[7]);
    } else {
      // hi + residual: x - hi is exact in FP32 (at most 13 significant bits)
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        uint16_t h[2], l[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float x = ldexpf((float)wacc[k0 + e + q], -eb);
          if (MODE == W_BF16) {
            h[q] = bf16_rne(x);
            l[q] = bf16_rne(x - bf16_to_f(h[q]));
          } else {
            h[q] = f16_rne(x);
            l[q] = f16_rne(x - f16_to_f(h[q]));
          }
        }
        hw[e >> 1] = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        lw[e >> 1] = (uint32_t)l[0] | ((uint32_t)l[1] << 16);
        on = on || (hw[e >> 1] | lw[e >> 1]) != 0u;
      }
      // eight consecutive entries of one row are contiguous in the fragment-tiled planes
      const size_t p = w16_pos(r, k0, K_pad >> 6);
      *(uint4 *)((uint16_t *)a.W + p) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *(uint4 *)((uint16_t *)a.Wlo + p) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
    const unsigned long long bal = __ballot(on);
    if (lane == 0) {
      const int c0 = c;               // lane 0 holds the wave's first run
      uint32_t bits = 0u;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if ((bal >> (4 * i)) & 0xfull) bits |= 1u << i;
      if (bits) atomicOr(&s_bits[c0 >> 7], bits << ((c0 >> 2) & 31));
    }
  }
  __syncthreads();
  for (int w = tid; w < a.mask_words; w += 256) a.rowmask[(size_t)r * a.mask_words + w] = s_bits[w];

  if (tid == 0) {
    PointRow pr;
    pr.z = z;
    pr.t_univ = s_tu;
    pr.dc = dc;
    pr.dl = (1.0 + z) * dc;
    pr.mass10 = s_m10;
    pr.scale_fnu = pr.mass10 * (1.0 + z) / (4.0 * kPi * pr.dl * pr.dl) * kLsun * kAng_cm / kC_cms;
    pr.wscale = wscale;
    pr.tau_bc = s_th[TH_TAU_BC];
    pr.alpha_bc = s_th[TH_ALPHA_BC];
    pr.tau_diff = s_th[TH_TAU_DIFF];
    pr.delta = s_th[TH_DELTA];
    pr.bc_p = bc_p;
    pr.bc_q = bc_q;
    pr.neb_s = neb_s;
    pr.fob = fob;
    pr.nc_j[0] = pr.nc_j[1] = 0;
    pr.nc_t[0] = pr.nc_t[1] = 0.0;
    if (lib.has_cont) {
      bool in;
      grid_split_dev(lib.cz, lib.n_cz, s_th[TH_GAS_LOGZ], pr.nc_j[0], pr.nc_t[0], in);
      grid_split_dev(lib.cu, lib.n_cu, s_th[TH_GAS_LOGU], pr.nc_j[1], pr.nc_t[1], in);
    }
    pr.b = b;
    pr.obs = slot;
    pr.kind = kind;
    pr.seg0 = 0;
    pr.seg_n = 0;
    if (lib.log_uniform) {
      if (kind == 0) phot_span(lib, fw_min, fw_max, z, pr.seg0, pr.seg_n);
      else if (kind == 1) spec_span(lib, px_lo, px_hi, ks_max, z, pr.seg0, pr.seg_n);
    }
    pr.cov0 = pr.seg0;
    pr.cov_n = pr.seg_n;
    if (lib.vdisp && vd_n > 0 && (kind == 0 || kind == 1)) vdisp_window(lib, vd_lo, vd_hi, vd_M, vd_dl, z, pr.cov0, pr.cov_n);
    a.rows[r] = pr;
  }
}

// ---------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------
size_t prep_smem_bytes(const DevLib &lib, int mode) {
  return sizeof(double) * (size_t)PrepSmem(lib, mode).total;
}

hipError_t launch_keys(const DevLib &lib, const double *theta, int P, int B, double *keys, int *ranks,
                       hipStream_t s) {
  if (!ranks && B <= kSelfKeyMaxB) return hipSuccess;   // the weight builder forms the keys itself
  hipLaunchKernelGGL(k_keys, dim3((B + 255) / 256), dim3(256), 0, s, lib, theta, P, B, keys);
  if (ranks) hipLaunchKernelGGL(k_rank, dim3((B + 63) / 64), dim3(256), 0, s, keys, B, ranks);
  return hipGetLastError();
}

hipError_t launch_prep(const DevLib &lib, const PrepLaunch &pl, hipStream_t s) {
  PrepArgs a;
  a.theta = pl.theta;
  a.keys = pl.keys;
  a.ranks = pl.ranks;
  a.P = pl.P;
  a.B = pl.B;
  a.B_pad = pl.B_pad;
  a.obs_table = pl.obs_table;
  a.point_obs = pl.point_obs;
  a.W = pl.W;
  a.Wlo = pl.Wlo;
  a.rowmask = pl.rowmask;
  a.mask_words = pl.mask_words;
  a.rows = pl.rows;
  a.Lline = pl.Lline;
  a.WQ = pl.WQ;
  a.kpos = pl.kpos;
  a.line_k0 = pl.line_k0;
  const size_t sm = prep_smem_bytes(lib, pl.mode);
  if (sm > 160 * 1024) return hipErrorInvalidValue;
  static size_t attr_set[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const void *fn[8] = {(const void *)k_prep<W_F64, false>, (const void *)k_prep<W_F32, false>,
                       (const void *)k_prep<W_BF16, false>, (const void *)k_prep<W_F16, false>,
                       (const void *)k_prep<W_F64, true>,  (const void *)k_prep<W_F32, true>,
                       (const void *)k_prep<W_BF16, true>,  (const void *)k_prep<W_F16, true>};
  const int md = (pl.mode & 3) + (lib.sfh_scheme == 1 ? 4 : 0);
  if (sm > 48 * 1024 && sm > attr_set[md]) {
    hipError_t e = hipFuncSetAttribute(fn[md], hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    attr_set[md] = sm;
  }
  void *args[2] = {(void *)&lib, (void *)&a};
  return hipLaunchKernel(fn[md], dim3(pl.B_pad), dim3(256), args, sm, s);
}


}  // namespace sps
