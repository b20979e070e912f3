// 16-bit library contraction with FP32 accumulation (BF16 or FP16 MFMA).
// The library row k is stored as 2^{e_k} (H_k + R_k) and the weight row of point b
// as 2^{e_b} 2^{-e_k} (W_h + W_l), both 16-bit hi + residual pairs (the weight planes
// in the fragment-tiled layout written by the weight builder).  The products
// W_h H (main pass), W_h R and W_l H (one refinement pass over the residual terms)
// accumulate into one FP32 accumulator; the dropped W_l R term is second order.  The
// reduced variants take W_h H alone, W_h H + W_h R, or W_h H + W_l H.
#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"

namespace sps {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct ContractArgs16 {
  const uint16_t *Wh, *Wl, *H, *R;
  int K_pad, N_pad;
  const uint32_t *rowmask;   // [B_pad][mask_words] occupancy bits of 32-wide K tiles
  int mask_words, n_tiles32, young_tiles32;
  unsigned long long *counter;
  const PointRow *rows;
  const float *lnlv, *da, *dd;
  float *F;
  const int *list;   // SPAN: the (M tile, N tile) pairs to compute (k_tile_list)
  // escape geometry: K ranges left out below / at and above the Lyman limit (pixel
  // ion_nlim); pass 1 adds the picket fence's dust-free part f_ob (young stars + ionising)
  TileSkip skip_lo, skip_hi;
  int ion_nlim, pass;
};

template <bool BF, int PASSES>
__device__ __forceinline__ v16f mfma16(const u32x4 &a, const u32x4 &b, v16f c) {
  if constexpr (BF) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  }
}

// Birth-cloud transmission p e^{-tau_BC} + q applied to the young-part accumulator.
template <int BM, int BN, int WTM>
__device__ __forceinline__ void bc16(v16f (&acc)[BM][BN], const float (*sp)[8], const float *c_lnlv, int wm, int lh) {
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = wm * WTM + i * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
      for (int j = 0; j < BN; ++j)
        acc[i][j][e] *= sp[rl][6] * expf(-sp[rl][0] * expf(sp[rl][1] * c_lnlv[j])) + sp[rl][7];
    }
}

// PASSES: 1 = W_h H; 2 = W_h H + W_h R; 3 = W_h H + W_h R + W_l H; 4 = W_h H + W_l H.
// Block tile MT (points: 128, or 64 for small batches) x 64 (wavelengths), K tile 64;
// MT / 32 waves stacked along M, each 32 x 64 (two 32x32x16 MFMA accumulators).  A row's
// sums do not depend on MT: the K tiles its M tile adds beyond its own are zero rows.  Each wave reads its own weight
// fragments straight from global memory into registers (the weight planes are stored
// fragment-tiled, so one wave load is two contiguous 512-byte runs) with two register
// sets, the next K tile in flight while the current one is multiplied.  The library
// tile is shared by the four waves through double-buffered LDS: one barrier per K tile.
// LDS rows are unpadded with the 16-byte chunks XOR-swizzled: chunk c of row r sits at
// c ^ (r & 7) ^ ((r >> 3) & 1), which keeps 16-byte reads of 8 consecutive rows, and of
// the 8 rows of one parity among 16 consecutive rows, on distinct banks.
// SPAN: the block's tile comes from the compacted list of pairs that meet the rows' spans
// (blocks past the list return at once); otherwise every pair of the grid.
template <bool BF, int PASSES, bool SPAN, int MT>
__global__ void __launch_bounds__(2 * MT, MT == 64 && (PASSES == 2 || PASSES == 3) ? 2 : 3) k_contract_16(ContractArgs16 a) {
  constexpr int NT = 64, KT = 64, NCH = KT / 8, WTM = 32, BM = 1, BN = 2, NTH = 2 * MT;
  constexpr bool USE_WL = PASSES >= 3, USE_R = PASSES == 2 || PASSES == 3;
  constexpr int B8 = NT * KT / 8 / NTH;   // 16-byte library chunks per thread and K tile
  __shared__ __attribute__((aligned(16))) uint16_t Bh[2][NT * KT];
  __shared__ __attribute__((aligned(16))) uint16_t Br[2][USE_R ? NT * KT : 8];
  __shared__ float sp[MT][8];
#define SPS_SW(r_, c_) ((r_) * KT + (((c_) ^ ((r_) & 7) ^ (((r_) >> 3) & 1)) << 3))

  const int n_nt = a.N_pad / NT;
  int mt, nt;
  if constexpr (SPAN) {
    if (!span_block_tile(a.list, mt, nt)) return;
  } else {
    balanced_tile(gridDim.x / n_nt, n_nt, 3, mt, nt);
  }
  const int m0 = mt * MT, n0 = nt * NT;
  const int tid = threadIdx.x, lane = tid & 63, wm = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int K_pad = a.K_pad, n_kt = K_pad / KT;

  for (int r = tid; r < MT; r += NTH) {
    const PointRow &pr = a.rows[m0 + r];
    sp[r][0] = (float)pr.tau_bc;
    sp[r][1] = (float)pr.alpha_bc;
    sp[r][2] = (float)pr.tau_diff;
    sp[r][3] = (float)pr.delta;
    sp[r][4] = (float)(0.85 - 1.9 * pr.delta);
    sp[r][5] = (float)(a.pass ? pr.fob * pr.wscale : pr.wscale);
    sp[r][6] = (float)pr.bc_p;
    sp[r][7] = (float)pr.bc_q;
  }
  v16f acc[BM][BN];
#pragma unroll
  for (int j = 0; j < BN; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[0][j][e] = 0.f;

  __shared__ int tl[kMaxKTiles32 / 2];   // active 64-wide K tiles of this M tile
  __shared__ uint32_t s_or[64];
  __shared__ int s_n[2];
  int nact, ny;
  // pass 1 (no birth cloud): every tile counts as young, so the transmission never applies
  block_tile_list(a.rowmask, a.mask_words, m0, MT, 2, a.n_tiles32, a.pass ? a.n_tiles32 : a.young_tiles32, tl, s_or,
                  s_n, nact, ny, n0 >= a.ion_nlim ? a.skip_hi : a.skip_lo);
  if (tid == 0 && a.counter) atomicAdd(a.counter, (unsigned long long)nact);   // (M, K, N) tiles run
  // weight fragments of this wave's 32-row group: lane (li, lh) takes chunk lh*4 + s of
  // row li at MFMA step s (the same permutation of K as the library fragments below)
  const size_t wbase = (size_t)((m0 >> 5) + wm) * n_kt * (KT * 32) + (size_t)(lh * 4) * 256 + li * 8;
  int offB[B8];
#pragma unroll
  for (int q = 0; q < B8; ++q) {
    const int idx = tid + NTH * q;
    offB[q] = (n0 + idx / NCH) * K_pad + (idx % NCH) * 8;
  }
  u32x4 ah0[4], al0[USE_WL ? 4 : 1], ah1[4], al1[USE_WL ? 4 : 1], rbh[B8], rbr[USE_R ? B8 : 1];
#define SPS_LOADA(t_, H_, L_)                                                      \
  {                                                                                \
    const size_t o_ = wbase + (size_t)tl[min(t_, nact - 1)] * (KT * 32);           \
    _Pragma("unroll") for (int s = 0; s < 4; ++s) {                                \
      H_[s] = *(const u32x4 *)(a.Wh + o_ + s * 256);                               \
      if constexpr (USE_WL) L_[s] = *(const u32x4 *)(a.Wl + o_ + s * 256);         \
    }                                                                              \
  }
#define SPS_LOADB(t_)                                                              \
  {                                                                                \
    const int k0_ = tl[min(t_, nact - 1)] * KT;                                    \
    _Pragma("unroll") for (int q = 0; q < B8; ++q) {                               \
      rbh[q] = *(const u32x4 *)(a.H + (offB[q] + k0_));                            \
      if constexpr (USE_R) rbr[q] = *(const u32x4 *)(a.R + (offB[q] + k0_));       \
    }                                                                              \
  }
#define SPS_STOREB(buf_)                                                           \
  {                                                                                \
    _Pragma("unroll") for (int q = 0; q < B8; ++q) {                               \
      const int idx = tid + NTH * q, row = idx / NCH, c = idx % NCH;               \
      *(u32x4 *)(&Bh[buf_][SPS_SW(row, c)]) = rbh[q];                              \
      if constexpr (USE_R) *(u32x4 *)(&Br[buf_][SPS_SW(row, c)]) = rbr[q];         \
    }                                                                              \
  }
  // the passes are interleaved over the two independent accumulators
#define SPS_MMA(buf_, H_, L_)                                                      \
  {                                                                                \
    _Pragma("unroll") for (int s = 0; s < 4; ++s) {                                \
      const int ch = lh * 4 + s;                                                   \
      u32x4 fb[BN], fr[BN];                                                        \
      _Pragma("unroll") for (int j = 0; j < BN; ++j) {                             \
        fb[j] = *(const u32x4 *)(&Bh[buf_][SPS_SW(j * 32 + li, ch)]);              \
        if constexpr (USE_R) fr[j] = *(const u32x4 *)(&Br[buf_][SPS_SW(j * 32 + li, ch)]); \
      }                                                                            \
      _Pragma("unroll") for (int j = 0; j < BN; ++j) acc[0][j] = mfma16<BF, PASSES>(H_[s], fb[j], acc[0][j]); \
      if constexpr (USE_R) {                                                       \
        _Pragma("unroll") for (int j = 0; j < BN; ++j) acc[0][j] = mfma16<BF, PASSES>(H_[s], fr[j], acc[0][j]); \
      }                                                                            \
      if constexpr (USE_WL) {                                                      \
        _Pragma("unroll") for (int j = 0; j < BN; ++j) acc[0][j] = mfma16<BF, PASSES>(L_[s], fb[j], acc[0][j]); \
      }                                                                            \
    }                                                                              \
  }

  float c_lnlv[BN], c_a[BN], c_d[BN];
#pragma unroll
  for (int j = 0; j < BN; ++j) {
    const int col = n0 + j * 32 + li;
    c_lnlv[j] = a.lnlv[col];
    c_a[j] = a.da[col];
    c_d[j] = a.dd[col];
  }
  if (nact > 0) {
    SPS_LOADB(0);
    SPS_LOADA(0, ah0, al0);
    SPS_STOREB(0);
    SPS_LOADB(1);
  }
  __syncthreads();
  // two K tiles per trip, so the two weight register sets and LDS buffers alternate
  // without copies; LDS buffer b is rewritten only after the barrier that follows its
  // last read.  Every prefetch is issued unconditionally (tile indices past the list
  // repeat its last tile and are never multiplied): with no loads under a branch the
  // waits on the memory counter cover exactly the tile about to be used, and the
  // prefetched tiles stay in flight across the multiply.
  for (int t = 0; t < nact; t += 2) {
    SPS_LOADA(t + 1, ah1, al1);
    if (t == ny) bc16<BM, BN, WTM>(acc, sp, c_lnlv, wm, lh);
    SPS_MMA(0, ah0, al0);
    SPS_STOREB(1);
    SPS_LOADB(t + 2);
    __syncthreads();
    if (t + 1 >= nact) break;
    SPS_LOADA(t + 2, ah0, al0);
    if (t + 1 == ny) bc16<BM, BN, WTM>(acc, sp, c_lnlv, wm, lh);
    SPS_MMA(1, ah1, al1);
    SPS_STOREB(0);
    SPS_LOADB(t + 3);
    __syncthreads();
  }
#undef SPS_LOADA
#undef SPS_LOADB
#undef SPS_STOREB
#undef SPS_MMA
#undef SPS_SW
  if (a.pass) {   // the picket fence's dust-free part, added to the attenuated sum
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = wm * WTM + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        float *f = a.F + (size_t)(m0 + rl) * a.N_pad + n0 + j * 32 + li;
        *f += acc[0][j][e] * sp[rl][5];
      }
    }
    return;
  }
  if (ny == nact) bc16<BM, BN, WTM>(acc, sp, c_lnlv, wm, lh);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int rl = wm * WTM + 8 * (e >> 2) + 4 * lh + (e & 3);
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int col = n0 + j * 32 + li;
      const float Td = expf(-sp[rl][2] * expf(sp[rl][3] * c_lnlv[j]) * (c_a[j] + sp[rl][4] * c_d[j]));
      a.F[(size_t)(m0 + rl) * a.N_pad + col] = acc[0][j][e] * Td * sp[rl][5];
    }
  }
}


template <bool BF, int PASSES>
static void launch16(const ContractArgs16 &a, int n_mt, int MT, int N_pad, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1) {
  const dim3 grid(n_mt * (N_pad / 64));
  if (MT == 64) {
    if (a.list) hipExtLaunchKernelGGL((k_contract_16<BF, PASSES, true, 64>), grid, dim3(128), 0, s, e0, e1, 0, a);
    else hipExtLaunchKernelGGL((k_contract_16<BF, PASSES, false, 64>), grid, dim3(128), 0, s, e0, e1, 0, a);
  } else {
    if (a.list) hipExtLaunchKernelGGL((k_contract_16<BF, PASSES, true, 128>), grid, dim3(256), 0, s, e0, e1, 0, a);
    else hipExtLaunchKernelGGL((k_contract_16<BF, PASSES, false, 128>), grid, dim3(256), 0, s, e0, e1, 0, a);
  }
}

hipError_t launch_contract16_impl(const DevLib &lib, const ContractLaunch &cl, int n_mt, hipStream_t s) {
  ContractArgs16 a;
  const int precision = cl.precision;
  const bool bf = precision == 2 || precision == 4 || precision == 6 || precision == 8;
  a.Wh = (const uint16_t *)cl.W;
  a.Wl = (const uint16_t *)cl.Wlo;
  a.H = bf ? lib.Hb : lib.Hh;
  a.R = bf ? lib.Rb : lib.Rh;
  a.K_pad = lib.K_pad;
  a.N_pad = lib.N_pad;
  a.rowmask = cl.rowmask;
  a.mask_words = cl.mask_words;
  a.n_tiles32 = lib.K_pad / kKTile;
  a.young_tiles32 = lib.K_young_pad / kKTile;
  a.counter = cl.counter;
  a.rows = cl.rows;
  a.lnlv = lib.lnlv_f;
  a.da = lib.dust_a_f;
  a.dd = lib.dust_d_f;
  a.F = (float *)cl.F;
  a.list = cl.list;
  a.pass = cl.pass;
  a.ion_nlim = lib.ion_nlim;
  a.skip_lo = escape_skip(lib, cl.pass, false);
  a.skip_hi = escape_skip(lib, cl.pass, true);
  const void *Yatt = cl.Yatt;
  // the gradient pass (which needs the young part) runs on the FP32 / FP64 paths only
  if (!a.H || !a.R || Yatt) return hipErrorInvalidValue;
  switch (precision) {
    case 2: launch16<true, 3>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 3: launch16<false, 3>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 4: launch16<true, 1>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 5: launch16<false, 1>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 6: launch16<true, 2>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 7: launch16<false, 2>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 8: launch16<true, 4>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    case 9: launch16<false, 4>(a, n_mt, cl.B_pad / n_mt, lib.N_pad, s, cl.ev_start, cl.ev_stop); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sps
