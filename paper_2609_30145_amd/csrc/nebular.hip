// Nebular continuum (App. C): for each point and model pixel, the sum over the nebular
// ages a of (sum_{alpha,m} W Q)_a 10^{Chat(a, lambda)}, Chat bilinear in (log Z_gas,
// log U) on the continuum cube (whose age axis the library load resampled, linearly in
// age, onto the SSP ages: with the bilinear step this is the cube's trilinear value),
// converted from L_nu per photon to Lsun/A, scaled by the escape geometry's covered
// fraction, sent through the young light's birth-cloud transmission and the diffuse
// screen, and added to the attenuated rest-frame spectrum F that the contraction wrote.
//
// Work per (point, pixel) is a loop over the nebular ages of four table reads, a bilinear
// combination, one exponential and an accumulation: VALU-bound.  A block of 16 waves
// takes one (M tile, 64-pixel N tile) pair of the contraction (the same compacted list
// when the launch is span-limited); lanes run along the pixels and the waves share out the
// tile's live rows (those whose own span reaches the N tile), so that a tile list of a
// few hundred pairs still puts several waves on every SIMD.
#include "common.h"
#include "kernels.h"

namespace sps {

struct NebArgs {
  int MT, n_nt;
  const PointRow *rows;
  const double *WQ;      // [B_pad][n_nc] photon-weighted masses / kWqScale
  void *F;
  const int *list;       // span-limited launch: the (M tile, N tile) pairs, else NULL
};

constexpr int kNebThreads = 1024;
constexpr int kNebWaves = kNebThreads / 64;
constexpr int kNebMaxAges = 128;   // nebular ages a library may carry (checked at load)
constexpr int kNebMaxMT = 128;
constexpr int kNebWqLds = 4096;    // FP32 masses staged in LDS when MT * ages fits
constexpr int kNebTabLds = 8192;   // FP32 cube columns staged per chunk (floats)
constexpr int kNebChunk = 8;       // at most this many ages per staged chunk
constexpr int kNebMaxPlanes = kNebTabLds / kSpanTile;   // (Z_gas, U) nodes (checked at load)
constexpr int kNebStage = kNebTabLds / 4 / kNebThreads;  // float4 per thread per chunk

template <typename T>
__global__ void __launch_bounds__(kNebThreads) k_nebc(DevLib lib, NebArgs a) {
  __shared__ __attribute__((aligned(16))) float s_tab[sizeof(T) == 4 ? kNebTabLds : 4];
  __shared__ float s_wq[sizeof(T) == 4 ? kNebWqLds : 1];   // [row][age] when MT * ages fits
  __shared__ int s_cor[kNebMaxMT][4];   // FP32: the row's four corner planes, as offsets in s_tab
  __shared__ int s_off[kNebMaxMT][4];   // FP64: the same as offsets in the cube
  __shared__ T s_w[kNebMaxMT][4];       // bilinear weights of the four corners
  __shared__ double s_par[kNebMaxMT][8];
  __shared__ int s_live[kNebMaxMT];
  __shared__ int s_order[kNebMaxMT];    // the live rows, compacted
  __shared__ int s_nlive;

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
  const int ncu = lib.n_cu, planes = lib.n_cz * ncu;
  const size_t slab = (size_t)planes * lib.N_pad;   // one nebular age of the cube
  const int ch = min(kNebChunk, kNebTabLds / (planes * kSpanTile));   // ages per staged chunk (FP32)
  const float *tabg = lib.cont_f + n0;
  // the FP32 table columns of one chunk of ages: two 16-byte loads per thread into
  // registers, then LDS (named registers and macros, so that nothing goes to scratch)
  static_assert(kNebStage == 2, "two staging registers per thread");
  float4 st0, st1;
#define SPS_NEB_SRC(i_, c0_)                                                                    \
  (tabg + (size_t)((c0_) + (i_) / ((kSpanTile / 4) * planes)) * slab +                          \
   (size_t)(((i_) / (kSpanTile / 4)) % planes) * lib.N_pad + 4 * ((i_) % (kSpanTile / 4)))
#define SPS_NEB_DST(i_) (s_tab + ((i_) / (kSpanTile / 4)) * kSpanTile + 4 * ((i_) % (kSpanTile / 4)))
#define SPS_NEB_LOAD(c0_)                                                                       \
  {                                                                                             \
    const int n4_ = min(ch, n_nc - (c0_)) * planes * (kSpanTile / 4);                           \
    st0 = *(const float4 *)SPS_NEB_SRC(min(tid, n4_ - 1), c0_);                                 \
    st1 = *(const float4 *)SPS_NEB_SRC(min(tid + kNebThreads, n4_ - 1), c0_);                   \
  }
#define SPS_NEB_STORE(c0_)                                                                      \
  {                                                                                             \
    const int n4_ = min(ch, n_nc - (c0_)) * planes * (kSpanTile / 4);                           \
    if (tid < n4_) *(float4 *)SPS_NEB_DST(tid) = st0;                                           \
    if (tid + kNebThreads < n4_) *(float4 *)SPS_NEB_DST(tid + kNebThreads) = st1;               \
  }
  // the first chunk and the tile's masses are in flight while the rows are set up
  if (sizeof(T) == 4) SPS_NEB_LOAD(0);
  const bool wq_lds = MT * n_nc <= kNebWqLds;
  static_assert(kNebWqLds == 4 * kNebThreads, "four staged masses per thread");
  double wq0 = 0.0, wq1 = 0.0, wq2 = 0.0, wq3 = 0.0;
  if (sizeof(T) == 4 && wq_lds) {
    const double *src = a.WQ + (size_t)m0 * n_nc;
    const int last = MT * n_nc - 1;
    wq0 = src[min(tid, last)];
    wq1 = src[min(tid + kNebThreads, last)];
    wq2 = src[min(tid + 2 * kNebThreads, last)];
    wq3 = src[min(tid + 3 * kNebThreads, last)];
  }
  // per row: live (a real point and, on span-limited launches, one whose projection reads
  // this N tile: its pixels [cov0, cov0 + cov_n) with the tile list's one-pixel margin),
  // the corners of its cell, the bilinear weights, the attenuation parameters
  if (tid < MT) {
    const int r = tid;
    const PointRow &pr = a.rows[m0 + r];
    bool live = pr.b >= 0;
    if (live && a.list && pr.cov_n > 0) live = pr.cov0 - 1 < n0 + kSpanTile && pr.cov0 + pr.cov_n + 1 > n0;
    s_live[r] = live;
    const int jz = pr.nc_j[0], ju = pr.nc_j[1];
    const double tz = pr.nc_t[0], tu = pr.nc_t[1];
    const int c00 = jz * ncu + ju, c01 = c00 + 1, c10 = c00 + ncu, c11 = c10 + 1;
    s_cor[r][0] = c00 * kSpanTile;
    s_cor[r][1] = c01 * kSpanTile;
    s_cor[r][2] = c10 * kSpanTile;
    s_cor[r][3] = c11 * kSpanTile;
    s_off[r][0] = c00 * lib.N_pad;
    s_off[r][1] = c01 * lib.N_pad;
    s_off[r][2] = c10 * lib.N_pad;
    s_off[r][3] = c11 * lib.N_pad;
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
  if (sizeof(T) == 4 && wq_lds) {
    const int nw = MT * n_nc;
    if (tid < nw) s_wq[tid] = (float)wq0;
    if (tid + kNebThreads < nw) s_wq[tid + kNebThreads] = (float)wq1;
    if (tid + 2 * kNebThreads < nw) s_wq[tid + 2 * kNebThreads] = (float)wq2;
    if (tid + 3 * kNebThreads < nw) s_wq[tid + 3 * kNebThreads] = (float)wq3;
  }
  if (sizeof(T) == 4) SPS_NEB_STORE(0);
  __syncthreads();
  // the live rows compacted in row order (a prefix count over the tile, read as LDS
  // broadcasts), so that the waves share them evenly
  if (tid < MT) {
    const int r = tid;
    int place = 0, n_live = 0;
    for (int j = 0; j < MT; ++j) {
      place += (j < r) & s_live[j];
      n_live += s_live[j];
    }
    if (s_live[r]) s_order[place] = r;
    if (r == 0) s_nlive = n_live;
  }
  __syncthreads();
  const int n_live = s_nlive, n = n0 + lane;
  constexpr int RPW = kNebMaxMT / kNebWaves;   // rows per wave at most

  if constexpr (sizeof(T) == 8) {
    // FP64: the table in log10 units, 10^x by exp10, read straight from the cube
    const double *tab = lib.cont_d + n;
    const double sc = lib.cont_sc_d[n], l = lib.lnlv_d[n], da = lib.dust_a_d[n], dd = lib.dust_d_d[n];
    double *F = (double *)a.F;
    for (int p = wv; p < n_live; p += kNebWaves) {
      const int r = s_order[p];
      const int o0 = s_off[r][0], o1 = s_off[r][1], o2 = s_off[r][2], o3 = s_off[r][3];
      const double w0 = s_w[r][0], w1 = s_w[r][1], w2 = s_w[r][2], w3 = s_w[r][3];
      const double *wq = a.WQ + (size_t)(m0 + r) * n_nc;
      double sum = 0.0;
      for (int q = 0; q < n_nc; ++q) {
        const double *t = tab + (size_t)q * slab;
        sum += wq[q] * exp10(w0 * t[o0] + w1 * t[o1] + w2 * t[o2] + w3 * t[o3]);
      }
      const double *pp = s_par[r];
      const double tbc = pp[5] * exp(-pp[0] * exp(pp[1] * l)) + pp[6];
      const double td = exp(-pp[2] * exp(pp[3] * l) * (da + pp[4] * dd));
      F[(size_t)(m0 + r) * lib.N_pad + n] += td * tbc * pp[7] * sc * sum;
    }
  } else {
    // FP32: the table in log2 units less a per-pixel reference (so every term is at most
    // one), 2^x by the hardware exponential.  The N tile's cube columns are staged in LDS
    // a chunk of ages at a time (the next chunk's loads in flight during the current one's
    // arithmetic); each wave accumulates its rows' sums in registers.
    float acc[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) acc[i] = 0.f;
    for (int c0 = 0; c0 < n_nc; c0 += ch) {
      const int nch = min(ch, n_nc - c0);
      const bool more = c0 + ch < n_nc;
      if (more) SPS_NEB_LOAD(c0 + ch);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int p = wv + kNebWaves * i;
        if (p < n_live) {   // the same row on every lane: uniform
          const int r = s_order[p];
          const int q0 = s_cor[r][0] + lane, q1 = s_cor[r][1] + lane, q2 = s_cor[r][2] + lane, q3 = s_cor[r][3] + lane;
          const float w0 = s_w[r][0], w1 = s_w[r][1], w2 = s_w[r][2], w3 = s_w[r][3];
          const float *wq = s_wq + r * n_nc + c0;
          const double *wqg = a.WQ + (size_t)(m0 + r) * n_nc + c0;
          float sum = 0.f;
#pragma unroll
          for (int u = 0; u < kNebChunk; ++u) {
            if (u < nch) {
              const float *t = s_tab + u * planes * kSpanTile;
              const float x = w0 * t[q0] + w1 * t[q1] + w2 * t[q2] + w3 * t[q3];
              sum += (wq_lds ? wq[u] : (float)wqg[u]) * __builtin_amdgcn_exp2f(x);
            }
          }
          acc[i] += sum;
        }
      }
      if (more) {
        __syncthreads();   // every wave is done with this chunk
        SPS_NEB_STORE(c0 + ch);
        __syncthreads();
      }
    }
    const float sc = lib.cont_sc_f[n], l = lib.lnlv_f[n], da = lib.dust_a_f[n], dd = lib.dust_d_f[n];
    float *F = (float *)a.F;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int p = wv + kNebWaves * i;
      if (p < n_live) {
        const int r = s_order[p];
        const double *pp = s_par[r];
        const float tbc = (float)pp[5] * expf(-(float)pp[0] * expf((float)pp[1] * l)) + (float)pp[6];
        const float td = expf(-(float)pp[2] * expf((float)pp[3] * l) * (da + (float)pp[4] * dd));
        F[(size_t)(m0 + r) * lib.N_pad + n] += td * tbc * (float)pp[7] * sc * acc[i];
      }
    }
  }
#undef SPS_NEB_SRC
#undef SPS_NEB_DST
#undef SPS_NEB_LOAD
#undef SPS_NEB_STORE
}

hipError_t launch_nebular(const DevLib &lib, const NebLaunch &nl, hipStream_t s) {
  if (!lib.has_cont) return hipSuccess;
  if (nl.MT > kNebMaxMT || nl.MT % 4 || lib.neb_a1 - lib.neb_a0 > kNebMaxAges || lib.n_cz * lib.n_cu > kNebMaxPlanes)
    return hipErrorInvalidValue;
  NebArgs a;
  a.MT = nl.MT;
  a.n_nt = lib.N_pad / kSpanTile;
  a.rows = nl.rows;
  a.WQ = nl.WQ;
  a.F = nl.F;
  a.list = nl.list;
  const dim3 grid((nl.B_pad / nl.MT) * a.n_nt);
  if (nl.f64) hipLaunchKernelGGL(k_nebc<double>, grid, dim3(kNebThreads), 0, s, lib, a);
  else hipLaunchKernelGGL(k_nebc<float>, grid, dim3(kNebThreads), 0, s, lib, a);
  return hipGetLastError();
}

}  // namespace sps
