// Library contraction F = T_d (T_BC * sum_young W L + sum_old W L) (eq. 1, eq. D2),
// fused with both attenuation factors.  The weight matrix is in young-first K order,
// so the birth-cloud transmission is applied to the accumulator once, between the
// young and the old K tiles; K tiles that are zero for every row of an M tile are
// skipped through the per-M-tile active list.
#include <hip/hip_ext.h>

#include <climits>

#include "common.h"
#include "kernels.h"

namespace sps {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct ContractArgs {
  const void *W, *Wlo;
  const void *LTa, *LTb;   // FP32/FP64: LTa; 16-bit: hi (LTa) and residual (LTb) planes
  int K_pad, N_pad, B_pad;
  const uint32_t *rowmask;   // [B_pad][mask_words] occupancy bits of 32-wide K tiles
  int mask_words, n_tiles32, young_tiles32;
  unsigned long long *counter;
  const PointRow *rows;
  const float *lnlv, *da, *dd;
  const double *lnlv_d, *da_d, *dd_d;
  void *F, *Yatt;
  const int *list;   // SPAN: the (M tile, N tile) pairs to compute (k_tile_list)
  // escape geometry: K ranges left out below / at and above the Lyman limit (pixel
  // ion_nlim); pass 1 adds the picket fence's dust-free part f_ob (young stars + ionising)
  TileSkip skip_lo, skip_hi;
  int ion_nlim, pass;
};

// blockIdx -> (m tile, n tile) for the FP32 / FP64 kernels: each XCD takes a contiguous
// range of (m, n) tiles with n fastest, so an XCD keeps its few M tiles of the weights
// in L2 while the library streams past (measured faster here than the column split
// used by the 16-bit kernel, whose weight tiles are half the size).
__device__ __forceinline__ void tile_of_block(int n_ntiles, int &mt, int &nt) {
  const int nblk = gridDim.x, bid = blockIdx.x;
  int logical = bid;
  if ((nblk & 7) == 0) logical = (bid & 7) * (nblk >> 3) + (bid >> 3);
  mt = logical / n_ntiles;
  nt = logical - mt * n_ntiles;
}

// ---------------------------------------------------------------------------------
// FP32: v_mfma_f32_32x32x2f32.  Lane (i = l & 31, h = l >> 5) feeds A[i][k] and
// B[k][i] with k = h*16 + s at MFMA step s, so each lane reads 16 contiguous
// floats of its LDS row per 32-wide K tile.
// ---------------------------------------------------------------------------------
template <int BM, int BN, int WTM, int WTN>
__device__ __forceinline__ void bc32(v16f (&acc)[BM][BN], const float (*sp)[8], const float *c_lnlv, const float *c_a,
                                     const float *c_d, float *Yatt, int N_pad, int m0, int n0, int wm, int wn, int li,
                                     int lh) {
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = wm * WTM + i * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        acc[i][j][e] *= sp[rl][5] * expf(-sp[rl][0] * expf(sp[rl][1] * c_lnlv[j])) + sp[rl][6];
        if (Yatt) {
          const float Td = expf(-sp[rl][2] * expf(sp[rl][3] * c_lnlv[j]) * (c_a[j] + sp[rl][4] * c_d[j]));
          const int col = n0 + wn * WTN + j * 32 + li;
          Yatt[(size_t)(m0 + rl) * N_pad + col] = acc[i][j][e] * Td;
        }
      }
    }
}

// Gradient pass: the attenuation factors in FP64 from FP64 row parameters and column
// tables, so that the model's band values (whose residuals the adjoint amplifies near the
// data) carry no FP32 rounding of large optical depths.
__device__ __forceinline__ void dust_f64(const double *spd, double l, double da, double dd, double &Tbc, double &Td) {
  Tbc = exp(-spd[0] * exp(spd[1] * l));
  Td = exp(-spd[2] * exp(spd[3] * l) * (da + spd[4] * dd));
}

template <int BM, int BN, int WTM, int WTN>
__device__ __forceinline__ void bc32p(double (&acc)[BM][BN][16], const double (*spd)[5], const double *c_l,
                                      const double *c_a, const double *c_d, float *Yatt, int N_pad, int m0, int n0,
                                      int wm, int wn, int li, int lh) {
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = wm * WTM + i * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        double Tbc, Td;
        dust_f64(spd[rl], c_l[j], c_a[j], c_d[j], Tbc, Td);
        acc[i][j][e] *= Tbc;
        if (Yatt) {
          const int col = n0 + wn * WTN + j * 32 + li;
          Yatt[(size_t)(m0 + rl) * N_pad + col] = (float)(acc[i][j][e] * Td);
        }
      }
    }
}

// PRECISE (gradient pass): each 32-wide K tile is accumulated in FP32 and the tile
// partials are summed in FP64.  SPAN: the block's tile comes from the compacted list of
// pairs that meet the rows' spans (blocks past the list return at once).
template <int MT, int NT, int WM, int WN, bool PRECISE, int MINW = 1, bool SPAN = false>
__global__ void __launch_bounds__(256, MINW) k_contract_f32(ContractArgs a) {
  constexpr int KT = 32, LDSK = KT + 4;
  constexpr int WTM = MT / WM, WTN = NT / WN, BM = WTM / 32, BN = WTN / 32;
  static_assert(WM * WN == 4, "4 waves");
  constexpr int A4 = MT * KT / 4 / 256, B4 = NT * KT / 4 / 256;
  __shared__ __attribute__((aligned(16))) float As[MT * LDSK];
  __shared__ __attribute__((aligned(16))) float Bs[NT * LDSK];
  __shared__ float sp[MT][8];
  __shared__ double spd[PRECISE ? MT : 1][5];

  int mt, nt;
  if constexpr (SPAN) {
    if (!span_block_tile(a.list, mt, nt)) return;
  } else {
    tile_of_block(a.N_pad / NT, mt, nt);
  }
  const int m0 = mt * MT, n0 = nt * NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 31, lh = lane >> 5;
  const float *W = (const float *)a.W;
  const float *LT = (const float *)a.LTa;
  const int K_pad = a.K_pad;

  for (int r = tid; r < MT; r += 256) {
    const PointRow &pr = a.rows[m0 + r];
    sp[r][0] = (float)pr.tau_bc;
    sp[r][1] = (float)pr.alpha_bc;
    sp[r][2] = (float)pr.tau_diff;
    sp[r][3] = (float)pr.delta;
    sp[r][4] = (float)(0.85 - 1.9 * pr.delta);
    sp[r][5] = (float)pr.bc_p;
    sp[r][6] = (float)pr.bc_q;
    sp[r][7] = (float)pr.fob;
    if constexpr (PRECISE) {
      spd[r][0] = pr.tau_bc;
      spd[r][1] = pr.alpha_bc;
      spd[r][2] = pr.tau_diff;
      spd[r][3] = pr.delta;
      spd[r][4] = 0.85 - 1.9 * pr.delta;
    }
  }

  v16f acc[BM][BN];
  double dacc[PRECISE ? BM : 1][PRECISE ? BN : 1][PRECISE ? 16 : 1];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        acc[i][j][e] = 0.f;
        if constexpr (PRECISE) dacc[i][j][e] = 0.0;
      }

  __shared__ int tl[kMaxKTiles32];
  __shared__ uint32_t s_or[64];
  __shared__ int s_n[2];
  int nact, ny;
  // pass 1 (no birth cloud): every tile counts as young, so the transmission never applies
  block_tile_list(a.rowmask, a.mask_words, m0, MT, 1, a.n_tiles32, a.pass ? a.n_tiles32 : a.young_tiles32, tl, s_or,
                  s_n, nact, ny, n0 >= a.ion_nlim ? a.skip_hi : a.skip_lo);
  if (threadIdx.x == 0 && a.counter) atomicAdd(a.counter, (unsigned long long)nact);   // (M, K, N) tiles run

  f32x4 ra[A4], rb[B4];
#define SPS_GLOAD32(t_)                                                              \
  {                                                                                  \
    const int k0_ = tl[min(t_, nact - 1)] * KT;                                      \
    _Pragma("unroll") for (int q = 0; q < A4; ++q) {                                 \
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;                   \
      ra[q] = *(const f32x4 *)(W + (size_t)(m0 + row) * K_pad + k0_ + c4 * 4);      \
    }                                                                                \
    _Pragma("unroll") for (int q = 0; q < B4; ++q) {                                 \
      const int idx = tid + 256 * q, row = idx >> 3, c4 = idx & 7;                   \
      rb[q] = *(const f32x4 *)(LT + (size_t)(n0 + row) * K_pad + k0_ + c4 * 4);     \
    }                                                                                \
  }

  // per-lane columns and their static factors
  float c_lnlv[BN], c_a[BN], c_d[BN];
  double c_l64[PRECISE ? BN : 1], c_a64[PRECISE ? BN : 1], c_d64[PRECISE ? BN : 1];
#pragma unroll
  for (int j = 0; j < BN; ++j) {
    const int col = n0 + wn * WTN + j * 32 + li;
    c_lnlv[j] = a.lnlv[col];
    c_a[j] = a.da[col];
    c_d[j] = a.dd[col];
    if constexpr (PRECISE) {
      c_l64[j] = a.lnlv_d[col];
      c_a64[j] = a.da_d[col];
      c_d64[j] = a.dd_d[col];
    }
  }

  __syncthreads();
  if (nact > 0) SPS_GLOAD32(0);
  for (int t = 0; t < nact; ++t) {
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
    SPS_GLOAD32(t + 1);   // unconditional (past the list: the last tile again, unused), so
                          // the memory-counter waits cover only the tile being stored
    if (t == ny) {
      if constexpr (PRECISE) {
        bc32p<BM, BN, WTM, WTN>(dacc, spd, c_l64, c_a64, c_d64, (float *)a.Yatt, a.N_pad, m0, n0, wm, wn, li, lh);
      } else {
        bc32<BM, BN, WTM, WTN>(acc, sp, c_lnlv, c_a, c_d, (float *)a.Yatt, a.N_pad, m0, n0, wm, wn, li, lh);
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
#pragma unroll
    for (int s = 0; s < 16; ++s)
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
    if constexpr (PRECISE) {
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            dacc[i][j][e] += (double)acc[i][j][e];
            acc[i][j][e] = 0.f;
          }
    }
  }
  if (!PRECISE && a.pass) {   // the picket fence's dust-free part, added to the attenuated sum
    float *F = (float *)a.F;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int rl = wm * WTM + i * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int col = n0 + wn * WTN + j * 32 + li;
          F[(size_t)(m0 + rl) * a.N_pad + col] += acc[i][j][e] * sp[rl][7];
        }
      }
    return;
  }
  if (ny == nact) {
    __syncthreads();
    if constexpr (PRECISE) {
      bc32p<BM, BN, WTM, WTN>(dacc, spd, c_l64, c_a64, c_d64, (float *)a.Yatt, a.N_pad, m0, n0, wm, wn, li, lh);
    } else {
      bc32<BM, BN, WTM, WTN>(acc, sp, c_lnlv, c_a, c_d, (float *)a.Yatt, a.N_pad, m0, n0, wm, wn, li, lh);
    }
  }
#undef SPS_GLOAD32

  // diffuse screen on everything and store
  float *F = (float *)a.F;
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = wm * WTM + i * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int col = n0 + wn * WTN + j * 32 + li;
        if constexpr (PRECISE) {
          double Tbc, Td;
          dust_f64(spd[rl], c_l64[j], c_a64[j], c_d64[j], Tbc, Td);
          F[(size_t)(m0 + rl) * a.N_pad + col] = (float)(dacc[i][j][e] * Td);
        } else {
          const float Td = expf(-sp[rl][2] * expf(sp[rl][3] * c_lnlv[j]) * (c_a[j] + sp[rl][4] * c_d[j]));
          F[(size_t)(m0 + rl) * a.N_pad + col] = acc[i][j][e] * Td;
        }
      }
    }
}

// ---------------------------------------------------------------------------------
// FP64 parity instance: LDS-tiled FMA, 64x64 tile, 4x4 outputs per thread.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_contract_f64(ContractArgs a) {
  constexpr int MT = 64, NT = 64, KT = 32, LDSK = KT + 1;
  __shared__ double As[MT * LDSK];
  __shared__ double Bs[NT * LDSK];
  __shared__ double sp[MT][8];
  int mt, nt;
  tile_of_block(a.N_pad / NT, mt, nt);
  const int m0 = mt * MT, n0 = nt * NT;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const double *W = (const double *)a.W;
  const double *LT = (const double *)a.LTa;
  for (int r = tid; r < MT; r += 256) {
    const PointRow &pr = a.rows[m0 + r];
    sp[r][0] = pr.tau_bc;
    sp[r][1] = pr.alpha_bc;
    sp[r][2] = pr.tau_diff;
    sp[r][3] = pr.delta;
    sp[r][4] = 0.85 - 1.9 * pr.delta;
    sp[r][5] = pr.bc_p;
    sp[r][6] = pr.bc_q;
    sp[r][7] = pr.fob;
  }
  double acc[4][4] = {};
  __shared__ int tl[kMaxKTiles32];
  __shared__ uint32_t s_or[64];
  __shared__ int s_n[2];
  int nact, ny;
  block_tile_list(a.rowmask, a.mask_words, m0, MT, 1, a.n_tiles32, a.pass ? a.n_tiles32 : a.young_tiles32, tl, s_or,
                  s_n, nact, ny, n0 >= a.ion_nlim ? a.skip_hi : a.skip_lo);
  if (threadIdx.x == 0 && a.counter) atomicAdd(a.counter, (unsigned long long)nact);   // (M, K, N) tiles run
  auto apply_bc = [&]() {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const int rl = ty + 16 * i, col = n0 + tx + 16 * j;
        const double T = sp[rl][5] * exp(-sp[rl][0] * exp(sp[rl][1] * a.lnlv_d[col])) + sp[rl][6];
        acc[i][j] *= T;
        if (a.Yatt) {
          const double Td = exp(-sp[rl][2] * exp(sp[rl][3] * a.lnlv_d[col]) * (a.da_d[col] + sp[rl][4] * a.dd_d[col]));
          ((double *)a.Yatt)[(size_t)(m0 + rl) * a.N_pad + col] = acc[i][j] * Td;
        }
      }
  };
  for (int t = 0; t < nact; ++t) {
    const int k0 = tl[t] * KT;
    __syncthreads();
    for (int idx = tid; idx < MT * KT; idx += 256) {
      const int row = idx / KT, c = idx % KT;
      As[row * LDSK + c] = W[(size_t)(m0 + row) * a.K_pad + k0 + c];
      Bs[row * LDSK + c] = LT[(size_t)(n0 + row) * a.K_pad + k0 + c];
    }
    __syncthreads();
    if (t == ny) apply_bc();
    for (int kk = 0; kk < KT; ++kk) {
      double av[4], bv[4];
      for (int i = 0; i < 4; ++i) av[i] = As[(ty + 16 * i) * LDSK + kk];
      for (int j = 0; j < 4; ++j) bv[j] = Bs[(tx + 16 * j) * LDSK + kk];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
  __syncthreads();
  double *F = (double *)a.F;
  if (a.pass) {   // the picket fence's dust-free part, added to the attenuated sum
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const int rl = ty + 16 * i, col = n0 + tx + 16 * j;
        F[(size_t)(m0 + rl) * a.N_pad + col] += acc[i][j] * sp[rl][7];
      }
    return;
  }
  if (ny == nact) apply_bc();
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int rl = ty + 16 * i, col = n0 + tx + 16 * j;
      const double Td = exp(-sp[rl][2] * exp(sp[rl][3] * a.lnlv_d[col]) * (a.da_d[col] + sp[rl][4] * a.dd_d[col]));
      F[(size_t)(m0 + rl) * a.N_pad + col] = acc[i][j] * Td;
    }
}

// ---------------------------------------------------------------------------------
// The tile list of a span-limited forward launch (common.h: span_block_tile).
// k_tile_span: one workgroup per M tile, one thread per row, the tile's span in N tiles
// from its rows' pixel spans (one pixel of margin each side) by a min / max reduction.
// k_tile_list, one workgroup: per-item counts (N tiles in N-tile-major order, M tiles
// otherwise), a block-wide exclusive scan, and the pairs written in order.
__global__ void __launch_bounds__(128) k_tile_span(const PointRow *__restrict__ rows, int MT, int n_nt,
                                                   int *__restrict__ spans) {
  __shared__ int s_lo[2], s_hi[2];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const PointRow &pr = rows[(size_t)blockIdx.x * MT + t];
  int lo = INT_MAX, hi = -1;
  if (pr.b >= 0 && pr.cov_n > 0) {
    lo = max(pr.cov0 - 1, 0) / kSpanTile;
    hi = min(pr.cov0 + pr.cov_n, n_nt * kSpanTile - 1) / kSpanTile;
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
  }
  if (lane == 0) {
    s_lo[wv] = lo;
    s_hi[wv] = hi;
  }
  __syncthreads();
  if (t == 0) {
    spans[2 * blockIdx.x] = MT > 64 ? min(s_lo[0], s_lo[1]) : s_lo[0];
    spans[2 * blockIdx.x + 1] = MT > 64 ? max(s_hi[0], s_hi[1]) : s_hi[0];
  }
}

// (spans == NULL: small batches, whose rows the list kernel reduces itself, one launch less)
__global__ void __launch_bounds__(256) k_tile_list(const PointRow *__restrict__ rows, const int *__restrict__ spans,
                                                   int B_pad, int MT, int n_nt, int nt_major, int *__restrict__ list) {
  __shared__ int lo[kTileListMaxM], hi[kTileListMaxM];
  __shared__ int s_wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n_mt = B_pad / MT;
  if (spans) {
    for (int m = tid; m < n_mt; m += 256) {
      lo[m] = spans[2 * m];
      hi[m] = spans[2 * m + 1];
    }
  } else {
    for (int m = tid; m < n_mt; m += 256) {
      lo[m] = INT_MAX;
      hi[m] = -1;
    }
    __syncthreads();
    // the 64 consecutive rows of a wave lie in one M tile (MT is 64 or 128): eight rows
    // per lane with their loads in flight, a wave reduction, one LDS atomic per wave and row
    // group (one pixel of margin each side of a row's span)
    for (int base = 0; base < B_pad; base += 256 * 8) {
      int b[8], c0[8], cn[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int r = min(base + 256 * q + tid, B_pad - 1);
        b[q] = rows[r].b;
        c0[q] = rows[r].cov0;
        cn[q] = rows[r].cov_n;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int r0 = base + 256 * q + wv * 64;
        if (r0 >= B_pad) break;
        int l = INT_MAX, h = -1;
        if (b[q] >= 0 && cn[q] > 0) {
          l = max(c0[q] - 1, 0) / kSpanTile;
          h = min(c0[q] + cn[q], n_nt * kSpanTile - 1) / kSpanTile;
        }
        for (int o = 32; o > 0; o >>= 1) {
          l = min(l, __shfl_xor(l, o));
          h = max(h, __shfl_xor(h, o));
        }
        if (lane == 0) {
          atomicMin(&lo[r0 / MT], l);
          atomicMax(&hi[r0 / MT], h);
        }
      }
    }
  }
  __syncthreads();
  const int n_items = nt_major ? n_nt : n_mt;
  auto count_of = [&](int i) {
    if (!nt_major) return hi[i] >= lo[i] ? hi[i] - lo[i] + 1 : 0;
    int c = 0;
    for (int m = 0; m < n_mt; ++m) c += (lo[m] <= i && i <= hi[m]) ? 1 : 0;
    return c;
  };
  const int chunk = (n_items + 255) / 256, i0 = min(tid * chunk, n_items), i1 = min(i0 + chunk, n_items);
  int mine = 0;
  for (int i = i0; i < i1; ++i) mine += count_of(i);
  int incl = mine;   // inclusive scan of the chunk counts: waves, then the four wave totals
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) s_wsum[wv] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wv; ++w) base += s_wsum[w];
  int off = base + incl - mine;
  for (int i = i0; i < i1; ++i) {
    if (nt_major) {
      for (int m = 0; m < n_mt; ++m)
        if (lo[m] <= i && i <= hi[m]) list[1 + off++] = (m << 16) | i;
    } else {
      for (int n = lo[i]; n <= hi[i]; ++n) list[1 + off++] = (i << 16) | n;
    }
  }
  if (tid == 0) list[0] = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
}

hipError_t launch_tile_list(const PointRow *rows, int B_pad, int MT, int n_nt, bool nt_major, int *list,
                            hipStream_t s) {
  if (B_pad / MT > kTileListMaxM || n_nt > 0xffff || (MT != 64 && MT != 128) || B_pad % MT) return hipErrorInvalidValue;
  // large batches: the M tiles' spans by a kernel of their own, stored after the largest
  // list these rows can make (tile_list_ints)
  int *spans = B_pad >= kRankKernelMinB ? list + 1 + (size_t)((B_pad + 63) / 64) * n_nt : nullptr;
  if (spans) hipLaunchKernelGGL(k_tile_span, dim3(B_pad / MT), dim3(MT), 0, s, rows, MT, n_nt, spans);
  hipLaunchKernelGGL(k_tile_list, dim3(1), dim3(256), 0, s, rows, spans, B_pad, MT, n_nt, nt_major ? 1 : 0, list);
  return hipGetLastError();
}

int contract_mtile(int precision, int B_pad) { return precision <= 1 || B_pad <= kSmallMtBatch ? 64 : 128; }
int contract_ktile_factor(int precision) { return precision >= 2 ? 2 : 1; }

hipError_t launch_contract16_impl(const DevLib &lib, const ContractLaunch &cl, int n_mt, hipStream_t s);

hipError_t launch_contract(const DevLib &lib, const ContractLaunch &cl, hipStream_t s) {
  ContractArgs a;
  a.W = cl.W;
  a.Wlo = cl.Wlo;
  a.K_pad = lib.K_pad;
  a.N_pad = lib.N_pad;
  a.B_pad = cl.B_pad;
  a.rowmask = cl.rowmask;
  a.mask_words = cl.mask_words;
  a.n_tiles32 = lib.K_pad / kKTile;
  a.young_tiles32 = lib.K_young_pad / kKTile;
  a.counter = cl.counter;
  a.rows = cl.rows;
  a.lnlv = lib.lnlv_f;
  a.da = lib.dust_a_f;
  a.dd = lib.dust_d_f;
  a.lnlv_d = lib.lnlv_d;
  a.da_d = lib.dust_a_d;
  a.dd_d = lib.dust_d_d;
  a.F = cl.F;
  a.Yatt = cl.Yatt;
  a.list = cl.list;
  a.pass = cl.pass;
  a.ion_nlim = lib.ion_nlim;
  a.skip_lo = escape_skip(lib, cl.pass, false);
  a.skip_hi = escape_skip(lib, cl.pass, true);
  const int MT = contract_mtile(cl.precision, cl.B_pad);
  const int n_mt = cl.B_pad / MT;
  if (cl.precision == 0) {
    a.LTa = lib.LT64;
    hipExtLaunchKernelGGL(k_contract_f64, dim3(n_mt * (lib.N_pad / 64)), dim3(256), 0, s, cl.ev_start, cl.ev_stop, 0,
                          a);
  } else if (cl.precision == 1) {
    a.LTa = lib.LT32;
    const dim3 grid(n_mt * (lib.N_pad / 64));
    if (cl.Yatt && cl.list)
      hipExtLaunchKernelGGL((k_contract_f32<64, 64, 2, 2, true, 2, true>), grid, dim3(256), 0, s, cl.ev_start,
                            cl.ev_stop, 0, a);
    else if (cl.Yatt)
      hipExtLaunchKernelGGL((k_contract_f32<64, 64, 2, 2, true, 2>), grid, dim3(256), 0, s, cl.ev_start, cl.ev_stop, 0,
                            a);
    else if (cl.list)
      hipExtLaunchKernelGGL((k_contract_f32<64, 64, 2, 2, false, 2, true>), grid, dim3(256), 0, s, cl.ev_start,
                            cl.ev_stop, 0, a);
    else
      hipExtLaunchKernelGGL((k_contract_f32<64, 64, 2, 2, false, 2>), grid, dim3(256), 0, s, cl.ev_start, cl.ev_stop,
                            0, a);
  } else {
    return launch_contract16_impl(lib, cl, n_mt, s);
  }
  return hipGetLastError();
}

}  // namespace sps
