// Nebular continuum (App. C): for each point and model pixel, the sum over the nebular
// ages a of (sum_{alpha,m} W Q)_a 10^{Chat(a, lambda)}, Chat bilinear in (log Z_gas,
// log U) on the continuum cube (whose age axis the library load resampled, linearly in
// age, onto the SSP ages: with the bilinear step this is the cube's trilinear value),
// converted from L_nu per photon to Lsun/A, scaled by the escape geometry's covered
// fraction, sent through the young light's birth-cloud transmission and the diffuse
// screen, and added to the attenuated rest-frame spectrum F that the contraction wrote.
//
// Work per (point, pixel) is a short loop of four table reads, a bilinear combination, one
// exponential and an accumulation per nebular age: VALU-bound.  A block takes one
// (M tile, 64-pixel N tile) pair of the contraction (the same compacted list when the
// launch is span-limited); lanes run along the pixels, so every table read of a wave is
// one contiguous 256-byte run, and the four waves split the M tile's rows.
#include "common.h"
#include "kernels.h"

namespace sps {

struct NebArgs {
  const double *theta;
  int P, MT, n_nt;
  const PointRow *rows;
  const double *WQ;      // [B_pad][n_nc] photon-weighted masses / kWqScale
  void *F;
  const int *list;       // span-limited launch: the (M tile, N tile) pairs, else NULL
};

constexpr int kNebMaxAges = 128;   // nebular ages a library may carry (checked at load)
constexpr int kNebMaxMT = 128;
constexpr int kNebWqLds = 4096;    // FP32 masses staged in LDS when MT * ages fits

template <typename T>
__global__ void __launch_bounds__(256) k_nebc(DevLib lib, NebArgs a) {
  __shared__ float s_wq[kNebWqLds];   // FP32 path, when the tile's masses fit: [row][age]
  __shared__ int s_off[kNebMaxMT][4];
  __shared__ T s_w[kNebMaxMT][4];
  __shared__ double s_par[kNebMaxMT][8];
  __shared__ int s_live[kNebMaxMT];
  const int MT = a.MT, n_nc = lib.neb_a1 - lib.neb_a0;
  int mt, nt;
  if (a.list) {
    if (!span_block_tile(a.list, mt, nt)) return;
  } else {
    mt = blockIdx.x / a.n_nt;
    nt = blockIdx.x - mt * a.n_nt;
  }
  const int m0 = mt * MT, n0 = nt * kSpanTile;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ncz = lib.n_cz, ncu = lib.n_cu;
  const size_t slab = (size_t)ncz * ncu * lib.N_pad;   // one nebular age of the cube
  // per row: the cell of (log Z_gas, log U) on the cube's axes, its four corner offsets and
  // bilinear weights, the attenuation parameters
  for (int r = tid; r < MT; r += 256) {
    const PointRow &pr = a.rows[m0 + r];
    const bool live = pr.b >= 0;
    s_live[r] = live;
    if (!live) continue;
    const double *th = a.theta + (size_t)pr.b * a.P;
    int jz = 0, ju = 0;
    double tz = 0.0, tu = 0.0;
    bool in;
    grid_split_dev(lib.cz, ncz, th[TH_GAS_LOGZ], jz, tz, in);
    grid_split_dev(lib.cu, ncu, th[TH_GAS_LOGU], ju, tu, in);
    s_off[r][0] = (jz * ncu + ju) * lib.N_pad;
    s_off[r][1] = (jz * ncu + ju + 1) * lib.N_pad;
    s_off[r][2] = ((jz + 1) * ncu + ju) * lib.N_pad;
    s_off[r][3] = ((jz + 1) * ncu + ju + 1) * lib.N_pad;
    s_w[r][0] = (T)((1.0 - tz) * (1.0 - tu));
    s_w[r][1] = (T)((1.0 - tz) * tu);
    s_w[r][2] = (T)(tz * (1.0 - tu));
    s_w[r][3] = (T)(tz * tu);
    s_par[r][0] = pr.tau_bc;
    s_par[r][1] = pr.alpha_bc;
    s_par[r][2] = pr.tau_diff;
    s_par[r][3] = pr.delta;
    s_par[r][4] = 0.85 - 1.9 * pr.delta;
    s_par[r][5] = pr.bc_p;
    s_par[r][6] = pr.bc_q;
    s_par[r][7] = pr.neb_s;
  }
  const bool wq_lds = MT * n_nc <= kNebWqLds;
  if (sizeof(T) == 4 && wq_lds) {
    for (int i = tid; i < MT * n_nc; i += 256) s_wq[i] = (float)a.WQ[(size_t)m0 * n_nc + i];
  }
  __syncthreads();
  const int n = n0 + lane;
  if (sizeof(T) == 8) {
    // FP64: the table in log10 units, 10^x by exp10; the per-row masses straight from
    // global memory (eight rows' worth staged at a time would not pay at this precision)
    const double *tab = lib.cont_d + n;
    const double sc = lib.cont_sc_d[n], l = lib.lnlv_d[n], da = lib.dust_a_d[n], dd = lib.dust_d_d[n];
    double *F = (double *)a.F;
    for (int r = wv; r < MT; r += 4) {
      if (!s_live[r]) continue;
      const int o0 = s_off[r][0], o1 = s_off[r][1], o2 = s_off[r][2], o3 = s_off[r][3];
      const double w0 = (double)s_w[r][0], w1 = (double)s_w[r][1], w2 = (double)s_w[r][2], w3 = (double)s_w[r][3];
      const double *wq = a.WQ + (size_t)(m0 + r) * n_nc;
      double sum = 0.0;
      for (int q = 0; q < n_nc; ++q) {
        const double *t = tab + (size_t)q * slab;
        sum += wq[q] * exp10(w0 * t[o0] + w1 * t[o1] + w2 * t[o2] + w3 * t[o3]);
      }
      const double *p = s_par[r];
      const double tbc = p[5] * exp(-p[0] * exp(p[1] * l)) + p[6];
      const double td = exp(-p[2] * exp(p[3] * l) * (da + p[4] * dd));
      F[(size_t)(m0 + r) * lib.N_pad + n] += td * tbc * p[7] * sc * sum;
    }
  } else {
    // FP32: the table in log2 units less a per-pixel reference (so every term is at most
    // one), 2^x by exp2f; four ages per trip with their 16 reads issued together
    const float *tab = lib.cont_f + n;
    const float sc = lib.cont_sc_f[n], l = lib.lnlv_f[n], da = lib.dust_a_f[n], dd = lib.dust_d_f[n];
    float *F = (float *)a.F;
    for (int r = wv; r < MT; r += 4) {
      if (!s_live[r]) continue;
      const int o0 = s_off[r][0], o1 = s_off[r][1], o2 = s_off[r][2], o3 = s_off[r][3];
      const float w0 = (float)s_w[r][0], w1 = (float)s_w[r][1], w2 = (float)s_w[r][2], w3 = (float)s_w[r][3];
      const float *wq = s_wq + r * n_nc;
      float wqr[4];
      const double *wqg = a.WQ + (size_t)(m0 + r) * n_nc;
      float sum = 0.f;
      int q = 0;
      for (; q + 4 <= n_nc; q += 4) {
        float v[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float *t = tab + (size_t)(q + u) * slab;
          v[u][0] = t[o0];
          v[u][1] = t[o1];
          v[u][2] = t[o2];
          v[u][3] = t[o3];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) wqr[u] = wq_lds ? wq[q + u] : (float)wqg[q + u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          sum += wqr[u] * exp2f(w0 * v[u][0] + w1 * v[u][1] + w2 * v[u][2] + w3 * v[u][3]);
      }
      for (; q < n_nc; ++q) {
        const float *t = tab + (size_t)q * slab;
        sum += (wq_lds ? wq[q] : (float)wqg[q]) * exp2f(w0 * t[o0] + w1 * t[o1] + w2 * t[o2] + w3 * t[o3]);
      }
      const double *p = s_par[r];
      const float tbc = (float)p[5] * expf(-(float)p[0] * expf((float)p[1] * l)) + (float)p[6];
      const float td = expf(-(float)p[2] * expf((float)p[3] * l) * (da + (float)p[4] * dd));
      F[(size_t)(m0 + r) * lib.N_pad + n] += td * tbc * (float)p[7] * sc * sum;
    }
  }
}

hipError_t launch_nebular(const DevLib &lib, const NebLaunch &nl, hipStream_t s) {
  if (!lib.has_cont) return hipSuccess;
  if (nl.MT > kNebMaxMT || lib.neb_a1 - lib.neb_a0 > kNebMaxAges) return hipErrorInvalidValue;
  NebArgs a;
  a.theta = nl.theta;
  a.P = lib.P;
  a.MT = nl.MT;
  a.n_nt = lib.N_pad / kSpanTile;
  a.rows = nl.rows;
  a.WQ = nl.WQ;
  a.F = nl.F;
  a.list = nl.list;
  const dim3 grid((nl.B_pad / nl.MT) * a.n_nt);
  if (nl.f64) hipLaunchKernelGGL(k_nebc<double>, grid, dim3(256), 0, s, lib, a);
  else hipLaunchKernelGGL(k_nebc<float>, grid, dim3(256), 0, s, lib, a);
  return hipGetLastError();
}

}  // namespace sps
