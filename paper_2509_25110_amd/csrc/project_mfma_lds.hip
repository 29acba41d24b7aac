// Wide-column projection product on the matrix cores, staged through LDS
// (gCAMB paper, Sec. 2.1 Eq. 2-3 per k: Delta_k[l][c] = sum_n J_k[l][n] S_k[n][c];
// the wide case is the batch, where every model that uses k adds 3 columns).
//
// Split-BF16x3 only: a = ah + al, b = bh + bl with ah = RNE_bf16(a),
// al = RNE_bf16(a - ah); a*b ~ ah*bh + ah*bl + al*bh on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the same arithmetic as the
// fragment-streaming kernel in project_mfma.hip, in the same order per
// 32-node block, so both give identical results).
//
// Workgroup: 512 threads (8 waves), tile 256 l rows x 128 columns; waves in
// a 4 (l) x 2 (columns) grid, each 64 x 64 = 4 x 4 MFMA blocks.  The tau axis
// advances in 32-node blocks; each block's J rows (FP32) and S columns (FP32)
// are loaded with 16-byte global loads, split into bf16 hi/lo once, and stored
// to LDS rows of 40 bf16 (80 bytes: the 16-byte fragment reads of 16
// consecutive rows then hit 16 distinct 4-bank groups).  Two LDS stages: the
// next block is fetched into registers while the current one is multiplied.
// Blocks above the Bessel band of the tile's first row (`top`) are skipped;
// J rows above `top` of a block are zero-filled on load (they were not
// written).  Workgroups are remapped so that consecutive tiles of one k row
// (which share its J rows and S columns) land on the same XCD and its L2.
#include "los_internal.hpp"

namespace los {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int TM = 256, TN = 128, KB = 32;
constexpr int LROW = 40;  // bf16 per LDS row (32 used + 8 pad)

struct Stage {
  u16 ah[TM * LROW], al[TM * LROW];
  u16 bh[TN * LROW], bl[TN * LROW];
};

__device__ inline void split_store(const float (&v)[8], u16 *hi, u16 *lo) {
  bf8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 x = (__bf16)v[e];
    h[e] = x;
    l[e] = (__bf16)(v[e] - (float)x);
  }
  *(bf8 *)hi = h;
  *(bf8 *)lo = l;
}

__global__ __launch_bounds__(512) void mfma_gemm_lds_kernel(GemmArgs a, int tiles_m, int tiles_n,
                                                            int kcount) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  Stage *st = (Stage *)smem;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, r16 = lane & 15;

  // XCD-aware work order: hardware gives workgroup L to XCD L % 8; work item
  // q = (L % 8) * per + L / 8 gives each XCD a contiguous range of items.
  // Items run column tile fastest, then l tile, then k row: the column tiles
  // that share one J tile follow each other, and an S column tile comes back
  // tiles_n items later, so both are re-read from that XCD's L2.
  const int64_t total = (int64_t)tiles_m * tiles_n * kcount;
  const int64_t L = blockIdx.x;
  const int64_t per = (total + 7) / 8;
  const int64_t q = (L % 8) * per + L / 8;
  if (q >= total) return;
  const int tn = (int)(q % tiles_n);
  const int tm = (int)((q / tiles_n) % tiles_m);
  const int ki = (int)(q / ((int64_t)tiles_m * tiles_n));

  const int64_t r = a.k0 + ki;
  const int ncol = a.col_cnt ? a.col_cnt[r] : a.ncol;
  const int c0 = tn * TN;
  if (c0 >= ncol) return;
  const int lb0 = tm * (TM / 16);  // first 16-row block of the tile
  int lb_last = a.nlb - 1;
  if (a.col_lmax) lb_last = min(lb_last, (a.col_lmax[a.col_off[r] + c0] - a.lmin) >> 4);
  if (lb0 > lb_last) return;  // whole workgroup: uniform

  const int64_t sbase = a.col_off ? a.col_off[r] * a.s_cstride : r * a.s_kstride;
  const int64_t dbase = a.col_off ? (a.col_off[r] - a.col_base) * (int64_t)a.nl
                                  : r * (int64_t)a.nl * ncol;
  const float *Jk = a.J + (int64_t)ki * a.nlp * a.ntp;
  const int *topk = a.top + (int64_t)ki * a.ntb;

  // load assignment: A rows (tid >> 1), nodes 16 * (tid & 1) .. +15;
  //                  B columns (tid >> 2), nodes 8 * (tid & 3) .. +7
  const int arow = tid >> 1, acol = 16 * (tid & 1);
  const int brow = tid >> 2, bcol = 8 * (tid & 3);
  const int a_blk = lb0 + (arow >> 4);
  const int64_t a_row_abs = (int64_t)lb0 * 16 + arow;
  const bool a_ok = a_blk <= lb_last && a_row_abs < a.nlp;
  const int bc = c0 + brow;
  const bool b_ok = bc < ncol;
  const float *bsrc = a.S + sbase + (int64_t)(b_ok ? bc : 0) * a.s_cstride;
  const bool b_vec = (a.s_cstride % 4 == 0) && (sbase % 4 == 0);

  float va[16], vb[8];
  auto fetch = [&](int tb) {
    const int top = topk[tb];
    const bool ok = a_ok && a_blk <= top;
    const float *src = Jk + a_row_abs * a.ntp + tb * KB + acol;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float4 x = ok ? *(const float4 *)(src + 4 * v) : float4{0.f, 0.f, 0.f, 0.f};
      va[4 * v] = x.x; va[4 * v + 1] = x.y; va[4 * v + 2] = x.z; va[4 * v + 3] = x.w;
    }
    const int n0 = tb * KB + bcol;
    if (b_ok && b_vec && n0 + 8 <= a.ntau) {
      const float4 x = *(const float4 *)(bsrc + n0);
      const float4 y = *(const float4 *)(bsrc + n0 + 4);
      vb[0] = x.x; vb[1] = x.y; vb[2] = x.z; vb[3] = x.w;
      vb[4] = y.x; vb[5] = y.y; vb[6] = y.z; vb[7] = y.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) vb[e] = (b_ok && n0 + e < a.ntau) ? bsrc[n0 + e] : 0.f;
    }
  };
  auto stash = [&](Stage &s) {
    const float (&a0)[8] = *(const float (*)[8])(va);
    const float (&a1)[8] = *(const float (*)[8])(va + 8);
    split_store(a0, s.ah + arow * LROW + acol, s.al + arow * LROW + acol);
    split_store(a1, s.ah + arow * LROW + acol + 8, s.al + arow * LROW + acol + 8);
    split_store(vb, s.bh + brow * LROW + bcol, s.bl + brow * LROW + bcol);
  };

  // wave tile: rows 64 * (w & 3) .., columns 64 * (w >> 2) ..
  const int wr = 64 * (w & 3), wc = 64 * (w >> 2);
  const int w_blk0 = lb0 + (wr >> 4);
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // first needed block
  int tb = 0;
  while (tb < a.ntb && topk[tb] < lb0) ++tb;
  if (tb < a.ntb) fetch(tb);
  int buf = 0;
  while (tb < a.ntb) {
    stash(st[buf]);
    __syncthreads();
    const int cur_top = min(topk[tb], lb_last);
    int nxt = tb + 1;
    while (nxt < a.ntb && topk[nxt] < lb0) ++nxt;
    if (nxt < a.ntb) fetch(nxt);
    // this wave's rows: blocks w_blk0 .. w_blk0 + 3; only those <= cur_top hold data
    const int nb = min(4, cur_top - w_blk0 + 1);
    if (nb > 0) {
      const Stage &s = st[buf];
      bf8 bh[4], bl[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wc + 16 * j + r16;
        bh[j] = *(const bf8 *)(s.bh + row * LROW + 8 * g);
        bl[j] = *(const bf8 *)(s.bl + row * LROW + 8 * g);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < nb) {
          const int row = wr + 16 * i + r16;
          const bf8 ah = *(const bf8 *)(s.ah + row * LROW + 8 * g);
          const bf8 al = *(const bf8 *)(s.al + row * LROW + 8 * g);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    buf ^= 1;
    tb = nxt;
  }

#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int blk = w_blk0 + i;
    if (blk > lb_last) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + wc + 16 * j + r16;
      if (c >= ncol) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = blk * 16 + 4 * g + v;
        if (row < a.nl) {
          const int64_t o = a.dtrans ? (int64_t)c * a.nl + row : (int64_t)row * ncol + c;
          a.delta[dbase + o] = acc[i][j][v];
        }
      }
    }
  }
}

}  // namespace

size_t gemm_lds_bytes() { return 2 * sizeof(Stage); }

hipError_t mfma_gemm_lds_launch(const GemmArgs &a, int kcount, int max_ncol, hipStream_t s) {
  const int tiles_m = (a.nlb * 16 + TM - 1) / TM;
  const int tiles_n = (max_ncol + TN - 1) / TN;
  const int64_t total = (int64_t)tiles_m * tiles_n * kcount;
  const int64_t grid = ((total + 7) / 8) * 8;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  // the LDS limit is a per-device function attribute: set once per device
  // (the batch first launches this kernel from its autotuner, outside capture)
  static bool attr_set[256] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  if (!attr_set[dev]) {
    e = hipFuncSetAttribute((const void *)mfma_gemm_lds_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes());
    if (e != hipSuccess) return e;
    attr_set[dev] = true;
  }
  hipLaunchKernelGGL(mfma_gemm_lds_kernel, dim3((unsigned)grid), dim3(512), gemm_lds_bytes(), s,
                     a, tiles_m, tiles_n, kcount);
  return hipGetLastError();
}

}  // namespace los
