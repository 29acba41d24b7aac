// Projection product with the Bessel tiles generated in LDS (gCAMB paper,
// Sec. 2.1 Eq. 2-3; per k the tau sum is Delta_k[l][c] = sum_n J_k[l][n] S_k[n][c]
// with J_k[l][n] = w_n j_l(k chi_n)), in two kernels per chunk of k rows:
//
// jseed_kernel (FP64, one lane per tau node): the node's top row R (below the
//   MFMA band cut ltop_mfma) and the pair w (j_R, j_{R+1}) (node_top_pair),
//   then ONE descending sweep that
//   leaves, at the top row of every 32-row segment at or below R, the pair
//   (w j_T, w j_{T+1}), T = min(R, segment top), in a seed table; also 1/x
//   and R per node and the largest R of every chunk of 64 nodes.  Nothing of
//   J itself is stored.
//
// fused_gemm_kernel (one workgroup per (k row, TM-row l tile, TN-column
//   tile)): the tau axis advances in chunks of 64 nodes, visiting only the
//   chunks whose largest R reaches the tile (two ballots over the chunk
//   table), and the sources, seeds and R of the next such chunk are loaded
//   while the matrix cores work on the current one.  Per chunk every
//   wave regenerates one 32-row segment of the l tile for the 64 nodes from
//   the seeds (FP64 recurrence in registers, one lane per node, rounded to
//   FP32 -- or split into bf16 hi/lo -- as it is written to LDS), the S
//   columns of the tile are staged in LDS, and the matrix cores multiply the
//   two.  The recurrence runs with the same coefficient cadence as the
//   Bessel-table kernel (coefficient (2l+1)/x formed exactly at the rows
//   16b + 15 and 16b + 7 above lmin, stepped by -2/x in between), so the
//   generated values are those of the table, and the products are
//   accumulated in the same order as the table-based kernels (32-node blocks
//   in increasing order; within a block the same fragment layout).
//
// Data per chunk row kc (workspace):
//   rtop[kc * ntp + n]                 R (absolute l) or -1 (no row in band)
//   nix[kc * ntp + n]                  1 / x (0 where R < 0)
//   seed[(kc * nseg + s) * ntp + n]    (w j_T, w j_{T+1}), T = min(R, lmin + 32 s + 31),
//                                      written for segments with lmin + 32 s <= R
//   cmax[kc * (ntp / 64) + c]          max of rtop over nodes 64 c .. 64 c + 63
// ntp = nodes padded to a multiple of 64 (at most 8192, so at most 128 chunks).
#include "bessel_dev.hpp"
#include "los_internal.hpp"

namespace los {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int KB = 64;  // tau nodes per LDS chunk

__device__ inline int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Smallest set bit >= from of the 128-bit mask (a1:a0), or -1.
__device__ inline int next_chunk(uint64_t a0, uint64_t a1, int from) {
  if (from < 64) {
    const uint64_t m = a0 & (~0ull << from);
    if (m) return __ffsll((unsigned long long)m) - 1;
    from = 64;
  }
  if (from < 128) {
    const uint64_t m = a1 & (~0ull << (from - 64));
    if (m) return 64 + __ffsll((unsigned long long)m) - 1;
  }
  return -1;
}

// ------------------------------------------------------------------ seeds

__global__ __launch_bounds__(256) void jseed_kernel(FusedArgs a) {
  const int ki = blockIdx.y;
  const int64_t i = a.row_index ? a.row_index[a.k0 + ki] : a.k0 + ki;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= a.ntp) return;
  int R = -1;
  double ix = 0.0, cur = 0.0, nxt = 0.0;
  if (n < a.ntau) {
    const double x = a.k[i] * (a.tau0 - a.tau[n]);
    const double wt = a.w[n];
    if (x >= kXTiny && wt != 0.0) {
      ix = 1.0 / x;
      R = node_top_pair(x, ix, wt, a.lmin, a.lmax, ltop_mfma_of(x), cur, nxt);
    }
  }
  // every lane of the wave is here (ntp is a multiple of 64): the wave's 64
  // nodes are chunk n / 64
  const int cm = wave_max_int(R);
  if ((threadIdx.x & 63) == 0) a.cmax[(int64_t)ki * (a.ntp / KB) + (n / KB)] = cm;
  const int64_t nb = (int64_t)ki * a.ntp + n;
  a.rtop[nb] = R;
  a.nix[nb] = R >= 0 ? ix : 0.0;
  if (R < 0) return;
  double2 *sd = a.seed + (int64_t)ki * a.nseg * a.ntp + n;
  const double d2 = ix + ix;
  // 16-row blocks b from R's block down to block 1; the pair at the top of
  // block b is stored when b is odd (a segment top) or b is R's own block.
  const int bR = (R - a.lmin) >> 4;
  for (int b = bR; b >= 1; --b) {
    if ((b & 1) || b == bR) sd[(int64_t)(b >> 1) * a.ntp] = make_double2(cur, nxt);
    if (b == 1) break;
    const int lbase = a.lmin + 16 * b;
    double t = 0.0;
#pragma unroll
    for (int r = 15; r >= 0; --r) {
      if (r == 15 || r == 7) t = (double)(2 * (lbase + r) + 1) * ix;
      const double pv = rec_step(t, cur, nxt);
      nxt = cur;
      cur = pv;
      t -= d2;
    }
  }
  if (bR == 0) sd[0] = make_double2(cur, nxt);
}

// ------------------------------------------------------------------ product

template <int PREC>
struct LdsLayout;
template <>
struct LdsLayout<1> {  // FP32 rows of KB + 4 floats (272 bytes: 16 consecutive rows hit 16 bank groups)
  static constexpr int LD = KB + 4;
  static constexpr size_t bytes(int tm, int tn) { return sizeof(float) * (size_t)(tm + tn) * LD; }
};
template <>
struct LdsLayout<2> {  // bf16 hi and lo rows of KB + 8 (144 bytes: 16 rows hit 16 bank groups)
  static constexpr int LD = KB + 8;
  static constexpr size_t bytes(int tm, int tn) { return 2 * sizeof(u16) * (size_t)(tm + tn) * LD; }
};

__device__ inline u16 bf16_bits(__bf16 v) { return __builtin_bit_cast(u16, v); }

// x rounded to FP32, as a value the compiler may not look through: the bf16
// split that follows must round this FP32 value (as the table pipeline does),
// not x itself (a direct FP64 -> bf16 rounding differs in rare ties).
__device__ inline float f32_opaque(double x) {
  float v = (float)x;
  asm("" : "+v"(v));
  return v;
}

// One LDS stage: the J tile [TM][LD] and the S tile [TN][LD] (FP32), or hi and
// lo copies of each (bf16), starting at byte offset `base` of the shared memory.
template <int PREC, int TM, int TN>
struct Stage {
  float *Jf, *Sf;
  u16 *Jh, *Jl, *Sh, *Sl;
  __device__ Stage(unsigned char *base) {
    constexpr int LD = LdsLayout<PREC>::LD;
    Jf = (float *)base;
    Sf = Jf + TM * LD;
    Jh = (u16 *)base;
    Jl = Jh + TM * LD;
    Sh = Jl + TM * LD;
    Sl = Sh + TN * LD;
  }
};

// A workgroup's tile: XCD x = L % 8 takes the rows of rank x, x + 8, ...
// (rank 0 = largest k, the most work); within a row the l tiles of one column
// tile follow each other (they read the same S columns, kept in that XCD's L2).
struct Tile {
  int ki, tm, ncol, c0, lb0, lb_last, tile_lo, top_cap;
  int64_t r, sbase, dbase;
};

// The tile (k rank kr, l tile tm, column tile tn); false when it has nothing
// to compute (ki, r, tm, lb0 and tile_lo are set either way).
template <int TM, int TN>
__device__ inline bool tile_at(const FusedArgs &a, int kcount, int64_t kr, int tm, int tn, Tile &t) {
  t.tm = tm;
  t.ki = kcount - 1 - (int)kr;
  t.r = a.k0 + t.ki;
  t.lb0 = tm * (TM / 16);
  t.tile_lo = 16 * t.lb0;  // first row of the tile (l - lmin)
  t.ncol = a.col_cnt ? a.col_cnt[t.r] : a.ncol;
  t.c0 = tn * TN;
  t.sbase = a.col_off ? a.col_off[t.r] * a.s_cstride : t.r * a.s_kstride;
  t.dbase = a.col_off ? (a.col_off[t.r] - a.col_base) * (int64_t)a.nl
                      : t.r * (int64_t)a.nl * t.ncol;
  if (t.c0 >= t.ncol) return false;
  t.lb_last = a.nlb - 1;
  if (a.col_lmax) t.lb_last = min(t.lb_last, (a.col_lmax[a.col_off[t.r] + t.c0] - a.lmin) >> 4);
  if (t.lb0 > t.lb_last) return false;
  t.top_cap = 16 * t.lb_last + 15 - t.tile_lo;  // last tile row any column needs
  return true;
}

// The work item of this block: XCD x = L % 8 takes the rows of rank x, x + 8,
// ... (rank 0 = largest k, the most work); within a row the l tiles of one
// column tile follow each other (they read the same S columns, kept in that
// XCD's L2).
__device__ inline bool block_item(int tiles_m, int tiles_n, int kcount, int64_t &kr, int &tm,
                                  int &tn) {
  const int64_t per_row = (int64_t)tiles_m * tiles_n;
  const int64_t L = blockIdx.x;
  const int64_t q = L >> 3;
  kr = (L & 7) + 8 * (q / per_row);
  tm = (int)(q % per_row % tiles_m);
  tn = (int)(q % per_row / tiles_m);
  return kr < kcount;
}

template <int TM, int TN>
__device__ inline bool tile_of_block(const FusedArgs &a, int tiles_m, int tiles_n, int kcount,
                                     Tile &t) {
  int64_t kr;
  int tm, tn;
  if (!block_item(tiles_m, tiles_n, kcount, kr, tm, tn)) return false;
  return tile_at<TM, TN>(a, kcount, kr, tm, tn, t);
}

// Active chunks: those whose largest top row reaches the tile's first row, as
// a 128-bit mask (the same in every wave), and the lane's entries of the
// chunk table (chunk_top reads them back).
struct Chunks {
  int cm0, cm1;
  uint64_t act0, act1;
};

__device__ inline Chunks active_chunks(const FusedArgs &a, const Tile &t, int lane) {
  const int nch = (int)(a.ntp / KB);  // <= 128
  const int *cmr = a.cmax + (int64_t)t.ki * nch;
  const int thr = a.lmin + t.tile_lo;
  Chunks ch;
  ch.cm0 = lane < nch ? cmr[lane] : -1;
  ch.cm1 = lane + 64 < nch ? cmr[lane + 64] : -1;
  ch.act0 = __ballot(ch.cm0 >= thr);
  ch.act1 = __ballot(ch.cm1 >= thr);
  return ch;
}

// The last tile row that holds data in chunk c (its largest R, capped).
__device__ inline int chunk_top(const FusedArgs &a, const Tile &t, const Chunks &ch, int c) {
  const int cmax = __shfl(c < 64 ? ch.cm0 : ch.cm1, c & 63, 64);
  return __builtin_amdgcn_readfirstlane(min(cmax - a.lmin - t.tile_lo, t.top_cap));  // uniform
}

// The S tile [TN columns][KB nodes] moves in 16-byte pieces, NTH threads.
template <int TN, int NTH>
struct SPieces {
  static constexpr int SP = TN * KB / 4;
  static constexpr int SPT = (SP + NTH - 1) / NTH;  // per thread (the last round may be partial)
};

// One chunk's inputs as one producing thread holds them: R, seed pair and 1/x
// of the lane's node (for the wave's segment) and the thread's S pieces.
template <int SPT>
struct ChunkIn {
  int R = -1;
  double2 sd = make_double2(0.0, 0.0);
  double nx = 0.0;
  float4 sv[SPT];
};

// What a producing wave needs to regenerate its segment and stage S.
struct Producer {
  int seg_hi;         // l - lmin of the segment's top row
  bool seg_ok;        // the segment exists (sg < nseg)
  bool s_vec;         // S columns are 16-byte aligned
  int64_t rowb;       // chunk row offset in the per-node tables
  const double2 *seedp;
};

__device__ inline Producer producer_of(const FusedArgs &a, const Tile &t, int sg) {
  Producer p;
  p.seg_ok = sg < a.nseg;
  p.seg_hi = 32 * sg + 31;
  p.rowb = (int64_t)t.ki * a.ntp;
  p.seedp = a.seed + ((int64_t)t.ki * a.nseg + (p.seg_ok ? sg : 0)) * a.ntp;
  p.s_vec = (a.s_cstride % 4 == 0) && (t.sbase % 4 == 0) && (a.ntau % 4 == 0);
  return p;
}

template <int TN, int NTH>
__device__ inline void load_chunk_in(const FusedArgs &a, const Tile &t, const Producer &p, int c,
                                     int lane, int pt, ChunkIn<SPieces<TN, NTH>::SPT> &in) {
  constexpr int SP = SPieces<TN, NTH>::SP, SPT = SPieces<TN, NTH>::SPT;
  const int n = c * KB + lane;
  in.R = a.rtop[p.rowb + n];
  in.nx = a.nix[p.rowb + n];
  if (p.seg_ok) in.sd = p.seedp[n];  // read whatever the node's R; used only below R
  // A chunk wholly inside the tau grid with 16-byte aligned columns loads its
  // pieces as 16-byte vectors with no branch (columns past ncol read column 0
  // and are zeroed); the last, ragged chunk goes element by element.
  if (p.s_vec && (c + 1) * KB <= a.ntau) {  // uniform
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      if (SP % NTH != 0 && q * NTH + pt >= SP) break;
      const int e = (q * NTH + pt) * 4;  // element within [TN][KB]
      const int col = e / KB, nn = e % KB;
      const int cg = t.c0 + col;
      const float4 v = *(const float4 *)(a.S + t.sbase + (int64_t)(cg < t.ncol ? cg : 0) * a.s_cstride +
                                         c * KB + nn);
      in.sv[q] = cg < t.ncol ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  } else {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      if (SP % NTH != 0 && q * NTH + pt >= SP) break;
      const int e = (q * NTH + pt) * 4;
      const int col = e / KB, nn = e % KB;
      const int cg = t.c0 + col, ng = c * KB + nn;
      const float *src = a.S + t.sbase + (int64_t)(cg < t.ncol ? cg : 0) * a.s_cstride + ng;
      float t4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) t4[u] = (cg < t.ncol && ng + u < a.ntau) ? src[u] : 0.f;
      in.sv[q] = make_float4(t4[0], t4[1], t4[2], t4[3]);
    }
  }
}

// Regenerate the 32 rows of a segment (tile rows tr_base .. tr_base + 31) for
// the lane's node, zeros above its R.  No branch per row: a node live only in
// the lower 16-row block enters the recurrence there from its seed, and rows
// above a node's R run the recurrence on zeros.
template <int PREC, int TM, int TN, int SPT>
__device__ inline void gen_segment(const FusedArgs &a, const Producer &p, const ChunkIn<SPT> &in,
                                   int tr_base, int lane, const Stage<PREC, TM, TN> &sm) {
  constexpr int LD = LdsLayout<PREC>::LD;
  const int Rrel = in.R - a.lmin;                       // < 0 when the node has no row
  const bool liveA = in.R >= 0 && Rrel >= p.seg_hi;       // live through the upper 16 rows
  const bool liveB = in.R >= 0 && Rrel >= p.seg_hi - 16;  // live in the lower 16 rows
  const double ix = liveB ? in.nx : 0.0;
  const double d2 = ix + ix;
  double cur = liveA ? in.sd.x : 0.0, nxt = liveA ? in.sd.y : 0.0;
#pragma unroll
  for (int half = 1; half >= 0; --half) {
    if (half == 0) {
      cur = liveA ? cur : (liveB ? in.sd.x : 0.0);
      nxt = liveA ? nxt : (liveB ? in.sd.y : 0.0);
    }
    const int hi_row = p.seg_hi - 16 * (1 - half);  // l - lmin of the block's top row
    const int tr0 = tr_base + 16 * half;            // tile row of the block's bottom row
    double tt = 0.0;
#pragma unroll
    for (int rr = 15; rr >= 0; --rr) {
      if (rr == 15 || rr == 7) tt = (double)(2 * (a.lmin + hi_row - 15 + rr) + 1) * ix;
      const float v = PREC == 1 ? (float)cur : f32_opaque(cur);
      const double pv = rec_step(tt, cur, nxt);
      nxt = cur;
      cur = pv;
      tt -= d2;
      const int row = tr0 + rr;
      if (PREC == 1) {
        sm.Jf[row * LD + lane] = v;
      } else {
        const __bf16 h = (__bf16)v;
        sm.Jh[row * LD + lane] = bf16_bits(h);
        sm.Jl[row * LD + lane] = bf16_bits((__bf16)(v - (float)h));
      }
    }
  }
}

// The thread's S pieces into the stage (FP32, or split into bf16 hi and lo).
template <int PREC, int TM, int TN, int NTH>
__device__ inline void store_s(const ChunkIn<SPieces<TN, NTH>::SPT> &in, int pt,
                               const Stage<PREC, TM, TN> &sm) {
  constexpr int LD = LdsLayout<PREC>::LD;
  constexpr int SP = SPieces<TN, NTH>::SP, SPT = SPieces<TN, NTH>::SPT;
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    if (SP % NTH != 0 && q * NTH + pt >= SP) break;
    const int e = (q * NTH + pt) * 4;
    const int col = e / KB, nn = e % KB;
    if (PREC == 1) {
      *(float4 *)(sm.Sf + col * LD + nn) = in.sv[q];
    } else {
      const float v4[4] = {in.sv[q].x, in.sv[q].y, in.sv[q].z, in.sv[q].w};
      u16 hh[4], ll[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const __bf16 h = (__bf16)v4[u];
        hh[u] = bf16_bits(h);
        ll[u] = bf16_bits((__bf16)(v4[u] - (float)h));
      }
      *(uint2 *)(sm.Sh + col * LD + nn) = make_uint2(hh[0] | ((unsigned)hh[1] << 16),
                                                     hh[2] | ((unsigned)hh[3] << 16));
      *(uint2 *)(sm.Sl + col * LD + nn) = make_uint2(ll[0] | ((unsigned)ll[1] << 16),
                                                     ll[2] | ((unsigned)ll[3] << 16));
    }
  }
}

// Column blocks whose models stop below a row block skip its products: the
// last 16-row block (relative to the tile) that column block j of the wave
// needs, from the l_max of its first column (columns are ordered by l_max,
// largest first, within a row).
template <int NBW>
__device__ inline void column_limits(const FusedArgs &a, const Tile &t, int wc, int (&jlast)[NBW]) {
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    const int cj = t.c0 + wc * NBW * 16 + 16 * j;
    jlast[j] = __builtin_amdgcn_readfirstlane(  // uniform
        (a.col_lmax && cj < t.ncol) ? ((a.col_lmax[a.col_off[t.r] + cj] - a.lmin) >> 4) - t.lb0
                                    : (cj < t.ncol ? a.nlb - 1 - t.lb0 : -1));
  }
}

// One chunk's products for one multiplying wave: its row blocks are
// bi = bofs + BSTR * i of the tile (those with data: 16 bi <= top_tr), its
// column blocks wc * NBW + j; the two 32-node blocks of the chunk in
// increasing order.  Every accumulator sees its terms in the same order
// whichever wave owns it.
template <int PREC, int TM, int TN, int MBW, int NBW, int BSTR>
__device__ inline void mfma_chunk(f4 (&acc)[MBW][NBW], const int (&jlast)[NBW], int bofs, int wc,
                                  int top_tr, int g, int r16, const Stage<PREC, TM, TN> &sm) {
  constexpr int LD = LdsLayout<PREC>::LD;
  if (16 * bofs > top_tr) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kofs = 32 * h + 8 * g;
    if (PREC == 1) {
      float bfv[NBW][8];
#pragma unroll
      for (int j = 0; j < NBW; ++j) {
        const float *src = sm.Sf + (wc * NBW * 16 + 16 * j + r16) * LD + kofs;
        const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
        bfv[j][0] = u.x; bfv[j][1] = u.y; bfv[j][2] = u.z; bfv[j][3] = u.w;
        bfv[j][4] = v.x; bfv[j][5] = v.y; bfv[j][6] = v.z; bfv[j][7] = v.w;
      }
#pragma unroll
      for (int i = 0; i < MBW; ++i) {
        const int bi = bofs + BSTR * i;
        if (16 * bi <= top_tr) {
          const float *src = sm.Jf + (16 * bi + r16) * LD + kofs;
          const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
          const float af[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
          if (bi <= jlast[NBW - 1]) {  // every column block: accumulators in turn
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
              for (int j = 0; j < NBW; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[e], bfv[j][e], acc[i][j], 0, 0, 0);
          } else {
#pragma unroll
            for (int j = 0; j < NBW; ++j)
              if (bi <= jlast[j]) {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                  acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[e], bfv[j][e], acc[i][j],
                                                                   0, 0, 0);
              }
          }
        }
      }
    } else {
      bf8 bh[NBW], bl[NBW];
#pragma unroll
      for (int j = 0; j < NBW; ++j) {
        const int row = wc * NBW * 16 + 16 * j + r16;
        bh[j] = *(const bf8 *)(sm.Sh + row * LD + kofs);
        bl[j] = *(const bf8 *)(sm.Sl + row * LD + kofs);
      }
#pragma unroll
      for (int i = 0; i < MBW; ++i) {
        const int bi = bofs + BSTR * i;
        if (16 * bi <= top_tr) {
          const int row = 16 * bi + r16;
          const bf8 ah = *(const bf8 *)(sm.Jh + row * LD + kofs);
          const bf8 al = *(const bf8 *)(sm.Jl + row * LD + kofs);
          if (bi <= jlast[NBW - 1]) {  // every column block: accumulators in turn
#pragma unroll
            for (int j = 0; j < NBW; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < NBW; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < NBW; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
          } else {
#pragma unroll
            for (int j = 0; j < NBW; ++j)
              if (bi <= jlast[j]) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
              }
          }
        }
      }
    }
  }
}

// Accumulators to Delta: lane holds rows 4g + v of each 16-row block, column
// r16 of each column block.
template <int MBW, int NBW, int BSTR>
__device__ inline void store_acc(const FusedArgs &a, const Tile &t, const f4 (&acc)[MBW][NBW],
                                 int bofs, int wc, int g, int r16) {
#pragma unroll
  for (int i = 0; i < MBW; ++i) {
    const int blk = t.lb0 + bofs + BSTR * i;
    if (blk > t.lb_last) break;
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      const int cc = t.c0 + wc * NBW * 16 + 16 * j + r16;
      if (cc >= t.ncol) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = blk * 16 + 4 * g + v;
        if (row < a.nl) {
          const int64_t o = a.dtrans ? (int64_t)cc * a.nl + row : (int64_t)row * t.ncol + cc;
          a.delta[t.dbase + o] = acc[i][j][v];
        }
      }
    }
  }
}

// One workgroup per (k row, TM-row l tile, TN-column tile), WR x WC waves that
// all take every role in turn: per active chunk each wave regenerates one
// 32-row segment, the threads stage S, and after a barrier each wave
// multiplies its row blocks wr, wr + WR, ... (interleaved, so that the waves
// share a tile's partly filled upper blocks) by its column blocks; the next
// chunk's inputs load meanwhile.
template <int PREC, int WR, int WC, int MBW, int NBW>
__global__ __launch_bounds__(64 * WR * WC) void fused_gemm_kernel(FusedArgs a, int tiles_m,
                                                                  int tiles_n, int kcount) {
  constexpr int NT = 64 * WR * WC;
  constexpr int TM = WR * MBW * 16, TN = WC * NBW * 16;
  static_assert(TM / 32 == WR * WC, "one 32-row segment per wave");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  Tile t;
  if (!tile_of_block<TM, TN>(a, tiles_m, tiles_n, kcount, t)) return;  // uniform
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
  const int g = lane >> 4, r16 = lane & 15;
  const int wr = w % WR, wc = w / WR;
  const Stage<PREC, TM, TN> sm(smem);
  const Producer p = producer_of(a, t, t.tm * (TM / 32) + w);
  const Chunks ch = active_chunks(a, t, lane);

  f4 acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  int jlast[NBW];
  column_limits(a, t, wc, jlast);

  ChunkIn<SPieces<TN, NT>::SPT> in;
  int c = next_chunk(ch.act0, ch.act1, 0);
  if (c >= 0) load_chunk_in<TN, NT>(a, t, p, c, lane, tid, in);
  while (c >= 0) {
    const int top_tr = chunk_top(a, t, ch, c);
    if (p.seg_ok && 32 * w <= top_tr) gen_segment(a, p, in, 32 * w, lane, sm);
    store_s<PREC, TM, TN, NT>(in, tid, sm);
    __syncthreads();
    // the next active chunk's inputs are in flight while the matrix cores run
    const int cn = next_chunk(ch.act0, ch.act1, c + 1);
    if (cn >= 0) load_chunk_in<TN, NT>(a, t, p, cn, lane, tid, in);
    // FP32: the wave's products go ahead of the other workgroup's segment
    // generation on the SIMD (1 % on C4; nothing for split-BF16x3)
    if constexpr (PREC == 1) __builtin_amdgcn_s_setprio(1);
    mfma_chunk<PREC, TM, TN, MBW, NBW, WR>(acc, jlast, wr, wc, top_tr, g, r16, sm);
    if constexpr (PREC == 1) __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    c = cn;
  }
  store_acc<MBW, NBW, WR>(a, t, acc, wr, wc, g, r16);
}

// Sets the large-LDS limit of a kernel once per device (a per-device function
// attribute).
template <typename K>
hipError_t allow_lds(K kern, size_t lds, bool (&done)[64]) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (lds > 64 * 1024 && !done[dev]) {
    e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    done[dev] = true;
  }
  return hipSuccess;
}

int64_t fused_grid(const FusedArgs &a, int kcount, int max_ncol, int tm, int tn, int &tiles_m,
                   int &tiles_n) {
  tiles_m = (a.nlb * 16 + tm - 1) / tm;
  tiles_n = (max_ncol + tn - 1) / tn;
  return 8 * (((int64_t)kcount + 7) / 8) * tiles_m * tiles_n;
}

template <int PREC, int WR, int WC, int MBW, int NBW>
hipError_t launch_fused_t(const FusedArgs &a, int kcount, int max_ncol, hipStream_t s) {
  constexpr int TM = WR * MBW * 16, TN = WC * NBW * 16;
  int tiles_m, tiles_n;
  const int64_t grid = fused_grid(a, kcount, max_ncol, TM, TN, tiles_m, tiles_n);
  if (grid > 0x7fffffff || grid < 1) return hipErrorInvalidValue;
  const size_t lds = LdsLayout<PREC>::bytes(TM, TN);
  auto kern = fused_gemm_kernel<PREC, WR, WC, MBW, NBW>;
  static bool done[64] = {};
  hipError_t e = allow_lds(kern, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * WR * WC), lds, s, a, tiles_m,
                     tiles_n, kcount);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_fused_p(const FusedArgs &a, int shape, int kcount, int max_ncol,
                          hipStream_t s) {
  switch (shape) {
    case 0: return launch_fused_t<PREC, 4, 2, 4, 4>(a, kcount, max_ncol, s);  // 256 x 128
    case 1: return launch_fused_t<PREC, 2, 2, 4, 4>(a, kcount, max_ncol, s);  // 128 x 128
    case 2: return launch_fused_t<PREC, 2, 4, 8, 2>(a, kcount, max_ncol, s);  // 256 x 128
    case 3: return launch_fused_t<PREC, 2, 4, 8, 4>(a, kcount, max_ncol, s);  // 256 x 256
    case 4: return launch_fused_t<PREC, 8, 1, 2, 1>(a, kcount, max_ncol, s);  // 256 x 16
    case 5: return launch_fused_t<PREC, 4, 1, 2, 1>(a, kcount, max_ncol, s);  // 128 x 16
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

FusedShape fused_shape_at(int i) {
  static const FusedShape shapes[kFusedShapeCount] = {
      {256, 128}, {128, 128}, {256, 128}, {256, 256}, {256, 16}, {128, 16}};
  return shapes[i];
}

size_t fused_seed_bytes_per_row(int nseg, int64_t ntp) {
  return (size_t)ntp * (sizeof(int) + sizeof(double) + sizeof(double2) * (size_t)nseg) +
         sizeof(int) * (size_t)(ntp / KB);
}

void fused_workspace_at(FusedArgs &a, void *ws, int kcount) {
  char *p = (char *)ws;
  a.seed = (double2 *)p;
  p += sizeof(double2) * (size_t)a.nseg * a.ntp * kcount;
  a.nix = (double *)p;
  p += sizeof(double) * (size_t)a.ntp * kcount;
  a.rtop = (int *)p;
  p += sizeof(int) * (size_t)a.ntp * kcount;
  a.cmax = (int *)p;
}

hipError_t jseed_launch(const FusedArgs &a, int kcount, hipStream_t s) {
  dim3 grid((unsigned)((a.ntp + 255) / 256), (unsigned)kcount);
  hipLaunchKernelGGL(jseed_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t fused_gemm_launch(const FusedArgs &a, int prec, int shape, int kcount, int max_ncol,
                             hipStream_t s) {
  if (prec == 1) return launch_fused_p<1>(a, shape, kcount, max_ncol, s);
  if (prec == 2) return launch_fused_p<2>(a, shape, kcount, max_ncol, s);
  return hipErrorInvalidValue;
}

}  // namespace los
