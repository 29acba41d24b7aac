// Projection product with the Bessel tiles generated in LDS (gCAMB paper,
// Sec. 2.1 Eq. 2-3; per k the tau sum is Delta_k[l][c] = sum_n J_k[l][n] S_k[n][c]
// with J_k[l][n] = w_n j_l(k chi_n)), in two kernels per chunk of k rows:
//
// jseed_kernel (FP64, one lane per tau node): the node's top row R and the
//   pair w (j_R, j_{R+1}) (node_top_pair), then ONE descending sweep that
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
      R = node_top_pair(x, ix, wt, a.lmin, a.lmax, cur, nxt);
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

template <int PREC, int WR, int WC, int MBW, int NBW>
__global__ __launch_bounds__(64 * WR * WC) void fused_gemm_kernel(FusedArgs a, int tiles_m,
                                                                  int tiles_n, int kcount) {
  constexpr int NT = 64 * WR * WC;
  constexpr int TM = WR * MBW * 16, TN = WC * NBW * 16;
  constexpr int NSEG = TM / 32;
  static_assert(NSEG == WR * WC, "one 32-row segment per wave");
  constexpr int LD = LdsLayout<PREC>::LD;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  // Work item: XCD x = L % 8 takes the rows of rank x, x + 8, ... (rank 0 =
  // largest k, the most work); within a row the l tiles of one column tile
  // follow each other (they read the same S columns, kept in that XCD's L2).
  const int64_t per_row = (int64_t)tiles_m * tiles_n;
  const int64_t L = blockIdx.x;
  const int64_t q = L >> 3;
  const int64_t kr = (L & 7) + 8 * (q / per_row);
  if (kr >= kcount) return;
  const int tm = (int)(q % per_row % tiles_m);
  const int tn = (int)(q % per_row / tiles_m);
  const int ki = kcount - 1 - (int)kr;
  const int64_t r = a.k0 + ki;

  const int ncol = a.col_cnt ? a.col_cnt[r] : a.ncol;
  const int c0 = tn * TN;
  if (c0 >= ncol) return;
  const int lb0 = tm * (TM / 16);
  int lb_last = a.nlb - 1;
  if (a.col_lmax) lb_last = min(lb_last, (a.col_lmax[a.col_off[r] + c0] - a.lmin) >> 4);
  if (lb0 > lb_last) return;  // uniform
  const int tile_lo = 16 * lb0;                  // first row of the tile (l - lmin)
  const int top_cap = 16 * lb_last + 15 - tile_lo;  // last tile row any column needs

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, r16 = lane & 15;
  const int wr = w % WR, wc = w / WR;

  const int64_t sbase = a.col_off ? a.col_off[r] * a.s_cstride : r * a.s_kstride;
  const int64_t dbase = a.col_off ? (a.col_off[r] - a.col_base) * (int64_t)a.nl
                                  : r * (int64_t)a.nl * ncol;

  // LDS: J tile [TM][LD], S tile [TN][LD] (FP32), or hi and lo copies of each (bf16)
  float *Jf = (float *)smem;
  float *Sf = Jf + TM * LD;
  u16 *Jh = (u16 *)smem, *Jl = Jh + TM * LD;
  u16 *Sh = Jl + TM * LD, *Sl = Sh + TN * LD;

  // generation role: wave w regenerates segment sg (rows 32 w .. 32 w + 31 of the tile)
  const int sg = tm * NSEG + w;
  const bool seg_ok = sg < a.nseg;
  const int seg_hi = 32 * sg + 31;  // l - lmin of the segment's top row
  const int64_t rowb = (int64_t)ki * a.ntp;
  const double2 *seedp = a.seed + ((int64_t)ki * a.nseg + (seg_ok ? sg : 0)) * a.ntp;

  // S staging role: NT threads cover TN columns x 64 nodes in 16-byte pieces
  constexpr int SP = TN * KB / 4;           // float4 pieces per chunk
  constexpr int SPT = (SP + NT - 1) / NT;   // per thread (the last round may be partial)
  const bool s_vec = (a.s_cstride % 4 == 0) && (sbase % 4 == 0) && (a.ntau % 4 == 0);

  f4 acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // Column blocks whose models stop below a row block skip its products: the
  // last 16-row block (relative to the tile) that column block j of this wave
  // needs, from the l_max of its first column (columns are ordered by l_max,
  // largest first, within a row).
  int jlast[NBW];
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    const int cj = c0 + wc * NBW * 16 + 16 * j;
    jlast[j] = (a.col_lmax && cj < ncol) ? ((a.col_lmax[a.col_off[r] + cj] - a.lmin) >> 4) - lb0
                                         : (cj < ncol ? a.nlb - 1 - lb0 : -1);
  }

  // Active chunks: those whose largest top row reaches the tile's first row.
  const int nch = (int)(a.ntp / KB);  // <= 128
  const int *cmr = a.cmax + (int64_t)ki * nch;
  const int thr = a.lmin + tile_lo;
  const int cm0 = lane < nch ? cmr[lane] : -1;
  const int cm1 = lane + 64 < nch ? cmr[lane + 64] : -1;
  const uint64_t act0 = __ballot(cm0 >= thr), act1 = __ballot(cm1 >= thr);

  // Per-chunk inputs, loaded one active chunk ahead: R, seed pair and 1/x of
  // this lane's node, and this thread's pieces of the S tile.
  int Rn = -1;
  double2 sd = make_double2(0.0, 0.0);
  double nx = 0.0;
  float4 sv[SPT];
  auto load_chunk = [&](int c) {
    const int n = c * KB + lane;
    Rn = a.rtop[rowb + n];
    nx = a.nix[rowb + n];
    if (seg_ok) sd = seedp[n];  // read whatever the node's R; used only below R
#pragma unroll
    for (int p = 0; p < SPT; ++p) {
      if (SP % NT != 0 && p * NT + tid >= SP) break;
      const int e = (p * NT + tid) * 4;  // element within [TN][KB]
      const int col = e / KB, nn = e % KB;
      const int cg = c0 + col, ng = c * KB + nn;
      const float *src = a.S + sbase + (int64_t)(cg < ncol ? cg : 0) * a.s_cstride + ng;
      if (cg < ncol && s_vec && ng + 4 <= a.ntau) {
        sv[p] = *(const float4 *)src;
      } else {
        float t4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t4[u] = (cg < ncol && ng + u < a.ntau) ? src[u] : 0.f;
        sv[p] = make_float4(t4[0], t4[1], t4[2], t4[3]);
      }
    }
  };

  int c = next_chunk(act0, act1, 0);
  if (c >= 0) load_chunk(c);
  while (c >= 0) {
    const int cmax = __shfl(c < 64 ? cm0 : cm1, c & 63, 64);  // the chunk's largest R
    const int top_tr = min(cmax - a.lmin - tile_lo, top_cap);

    // regenerate this wave's segment for the 64 nodes (zeros above each node's R)
    if (seg_ok && 32 * w <= top_tr) {
      const int Rrel = Rn - a.lmin;                  // < 0 when the node has no row
      const bool liveA = Rn >= 0 && Rrel >= seg_hi;  // live through the upper 16 rows
      const bool liveB = Rn >= 0 && Rrel >= seg_hi - 16;
      double cur = liveB ? sd.x : 0.0, nxt = liveB ? sd.y : 0.0, ix = liveB ? nx : 0.0;
      const double d2 = ix + ix;
#pragma unroll
      for (int half = 1; half >= 0; --half) {
        const bool live = half ? liveA : liveB;
        const int hi_row = seg_hi - 16 * (1 - half);  // l - lmin of the block's top row
        const int tr0 = 32 * w + 16 * half;          // tile row of the block's bottom row
        double t = 0.0;
#pragma unroll
        for (int rr = 15; rr >= 0; --rr) {
          float v = 0.f;
          if (live) {
            if (rr == 15 || rr == 7) t = (double)(2 * (a.lmin + hi_row - 15 + rr) + 1) * ix;
            v = (float)cur;
            const double pv = rec_step(t, cur, nxt);
            nxt = cur;
            cur = pv;
            t -= d2;
          }
          const int row = tr0 + rr;
          if (PREC == 1) {
            Jf[row * LD + lane] = v;
          } else {
            const __bf16 h = (__bf16)v;
            Jh[row * LD + lane] = bf16_bits(h);
            Jl[row * LD + lane] = bf16_bits((__bf16)(v - (float)h));
          }
        }
      }
    }
    // S registers -> LDS
#pragma unroll
    for (int p = 0; p < SPT; ++p) {
      if (SP % NT != 0 && p * NT + tid >= SP) break;
      const int e = (p * NT + tid) * 4;
      const int col = e / KB, nn = e % KB;
      const float v4[4] = {sv[p].x, sv[p].y, sv[p].z, sv[p].w};
      if (PREC == 1) {
        *(float4 *)(Sf + col * LD + nn) = sv[p];
      } else {
        u16 hh[4], ll[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const __bf16 h = (__bf16)v4[u];
          hh[u] = bf16_bits(h);
          ll[u] = bf16_bits((__bf16)(v4[u] - (float)h));
        }
        *(uint2 *)(Sh + col * LD + nn) = make_uint2(hh[0] | ((unsigned)hh[1] << 16),
                                                   hh[2] | ((unsigned)hh[3] << 16));
        *(uint2 *)(Sl + col * LD + nn) = make_uint2(ll[0] | ((unsigned)ll[1] << 16),
                                                   ll[2] | ((unsigned)ll[3] << 16));
      }
    }
    __syncthreads();
    // the next active chunk's inputs are in flight while the matrix cores run
    const int cn = next_chunk(act0, act1, c + 1);
    if (cn >= 0) load_chunk(cn);

    // this wave's rows: blocks wr*MBW .. +MBW-1 of the tile; those <= top_tr hold data
    const int nb = min(MBW, (top_tr - wr * MBW * 16) / 16 + 1);
    if (top_tr >= wr * MBW * 16 && nb > 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {  // two 32-node blocks, in increasing order
        const int kofs = 32 * h + 8 * g;
        if (PREC == 1) {
          float bfv[NBW][8];
#pragma unroll
          for (int j = 0; j < NBW; ++j) {
            const float *src = Sf + (wc * NBW * 16 + 16 * j + r16) * LD + kofs;
            const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
            bfv[j][0] = u.x; bfv[j][1] = u.y; bfv[j][2] = u.z; bfv[j][3] = u.w;
            bfv[j][4] = v.x; bfv[j][5] = v.y; bfv[j][6] = v.z; bfv[j][7] = v.w;
          }
#pragma unroll
          for (int i = 0; i < MBW; ++i) {
            if (i < nb) {
              const float *src = Jf + (wr * MBW * 16 + 16 * i + r16) * LD + kofs;
              const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
              const float af[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
              if (wr * MBW + i <= jlast[NBW - 1]) {  // every column block: accumulators in turn
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                  for (int j = 0; j < NBW; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[e], bfv[j][e], acc[i][j],
                                                                     0, 0, 0);
              } else {
#pragma unroll
                for (int j = 0; j < NBW; ++j)
                  if (wr * MBW + i <= jlast[j]) {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[e], bfv[j][e],
                                                                       acc[i][j], 0, 0, 0);
                  }
              }
            }
          }
        } else {
          bf8 bh[NBW], bl[NBW];
#pragma unroll
          for (int j = 0; j < NBW; ++j) {
            const int row = wc * NBW * 16 + 16 * j + r16;
            bh[j] = *(const bf8 *)(Sh + row * LD + kofs);
            bl[j] = *(const bf8 *)(Sl + row * LD + kofs);
          }
#pragma unroll
          for (int i = 0; i < MBW; ++i) {
            if (i < nb) {
              const int row = wr * MBW * 16 + 16 * i + r16;
              const bf8 ah = *(const bf8 *)(Jh + row * LD + kofs);
              const bf8 al = *(const bf8 *)(Jl + row * LD + kofs);
              if (wr * MBW + i <= jlast[NBW - 1]) {  // every column block: accumulators in turn
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
                  if (wr * MBW + i <= jlast[j]) {
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
    __syncthreads();
    c = cn;
  }

  // output: lane holds rows 4g + v of each 16-row block, column r16 of each column block
#pragma unroll
  for (int i = 0; i < MBW; ++i) {
    const int blk = lb0 + wr * MBW + i;
    if (blk > lb_last) break;
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      const int cc = c0 + wc * NBW * 16 + 16 * j + r16;
      if (cc >= ncol) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = blk * 16 + 4 * g + v;
        if (row < a.nl) {
          const int64_t o = a.dtrans ? (int64_t)cc * a.nl + row : (int64_t)row * ncol + cc;
          a.delta[dbase + o] = acc[i][j][v];
        }
      }
    }
  }
}

template <int PREC, int WR, int WC, int MBW, int NBW>
hipError_t launch_fused_t(const FusedArgs &a, int kcount, int max_ncol, hipStream_t s) {
  constexpr int TM = WR * MBW * 16, TN = WC * NBW * 16;
  const int tiles_m = (a.nlb * 16 + TM - 1) / TM;
  const int tiles_n = (max_ncol + TN - 1) / TN;
  const int64_t grid = 8 * (((int64_t)kcount + 7) / 8) * tiles_m * tiles_n;
  if (grid > 0x7fffffff || grid < 1) return hipErrorInvalidValue;
  const size_t lds = LdsLayout<PREC>::bytes(TM, TN);
  auto kern = fused_gemm_kernel<PREC, WR, WC, MBW, NBW>;
  // the large-LDS limit is a per-device function attribute
  static bool attr_set[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (lds > 64 * 1024 && !attr_set[dev]) {
    e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    attr_set[dev] = true;
  }
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
