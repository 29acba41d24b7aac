// Projection as a matrix product on the matrix cores (gCAMB paper, Sec. 2.1
// Eq. 2-3; per k the sum over tau is Delta_k[l][c] = sum_n J_k[l][n] S_k[n][c]
// with J_k the weighted Bessel table from jtable.hip):
//
//   LOS_FP32   : v_mfma_f32_16x16x4_f32, FP32 inputs, FP32 accumulation;
//   LOS_BF16X3 : v_mfma_f32_16x16x32_bf16 on split operands a = ah + al,
//                b = bh + bl (ah = RNE_bf16(a), al = RNE_bf16(a - ah), the
//                subtraction exact in FP32); a*b ~ ah*bh + ah*bl + al*bh,
//                FP32 accumulation.  The al*bl term (< 2^-16 relative) is
//                dropped.
//
// Tiling: a workgroup is 4 waves; a wave owns MB consecutive 16-row l blocks
// and NC consecutive 16-column blocks and walks the tau axis in 32-node
// blocks, skipping every (l block, tau block) pair that lies above the
// Bessel band (the `top` table written with J).  Fragments come straight
// from global memory (J rows are re-read once per column tile, S columns
// once per l tile).
//
// Operand layout (one 32-node block, lane l, g = l / 16, e = 0..7):
//   A: row (l % 16) of the l block, nodes 8g + e;
//   B: column (l % 16) of the column block, nodes 8g + e.
// For the bf16 instruction this is its native 16x32 / 32x16 fragment; for the
// f32 instruction step e uses k index g <-> node 8g + e on both operands, so
// the 8 steps cover the same 32 nodes.  Output: lane l holds rows
// 4g + v (v = 0..3), column l % 16.
#include "los_internal.hpp"

namespace los {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct Frag {
  float v[8];
};

__device__ inline void split_bf16(const Frag &f, bf8 &hi, bf8 &lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)f.v[e];
    hi[e] = h;
    lo[e] = (__bf16)(f.v[e] - (float)h);
  }
}

template <int PREC, int MB, int NC>
__global__ __launch_bounds__(256) void mfma_gemm_kernel(GemmArgs a) {
  const int ki = blockIdx.z;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, r16 = lane & 15;
  const int64_t r = a.k0 + ki;
  const int lb0 = (blockIdx.x * 4 + w) * MB;
  if (lb0 >= a.nlb) return;
  const int ncol = a.col_cnt ? a.col_cnt[r] : a.ncol;
  const int cb0 = blockIdx.y * NC;
  if (cb0 * 16 >= ncol) return;
  // last 16-row block any column of this wave needs
  int lb_last = a.nlb - 1;
  if (a.col_lmax) lb_last = min(lb_last, (a.col_lmax[a.col_off[r] + cb0 * 16] - a.lmin) >> 4);
  if (lb0 > lb_last) return;

  const int64_t sbase = a.col_off ? a.col_off[r] * a.s_cstride : r * a.s_kstride;
  const int64_t dbase = a.col_off ? (a.col_off[r] - a.col_base) * (int64_t)a.nl
                                  : r * (int64_t)a.nl * ncol;
  const float *Jk = a.J + (int64_t)ki * a.nlp * a.ntp;
  const int *topk = a.top + (int64_t)ki * a.ntb;

  f4 acc[MB][NC];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int tb = 0; tb < a.ntb; ++tb) {
    const int top = min(topk[tb], lb_last);
    if (top < lb0) continue;
    const int nb = min(MB, top - lb0 + 1);
    const int n0 = tb * 32 + 8 * g;

    Frag bf[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = (cb0 + j) * 16 + r16;
      const float *src = a.S + sbase + (int64_t)c * a.s_cstride;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        bf[j].v[e] = (c < ncol && n0 + e < a.ntau) ? src[n0 + e] : 0.f;
    }
    Frag af[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      if (i < nb) {
        const float *src = Jk + (int64_t)((lb0 + i) * 16 + r16) * a.ntp + n0;
        const float4 u = *(const float4 *)src;
        const float4 v = *(const float4 *)(src + 4);
        af[i].v[0] = u.x; af[i].v[1] = u.y; af[i].v[2] = u.z; af[i].v[3] = u.w;
        af[i].v[4] = v.x; af[i].v[5] = v.y; af[i].v[6] = v.z; af[i].v[7] = v.w;
      }
    }

    if (PREC == 1) {
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (i < nb) {
#pragma unroll
          for (int j = 0; j < NC; ++j)
#pragma unroll
            for (int e = 0; e < 8; ++e)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].v[e], bf[j].v[e], acc[i][j],
                                                               0, 0, 0);
        }
      }
    } else {
      bf8 bh[NC], bl[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) split_bf16(bf[j], bh[j], bl[j]);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (i < nb) {
          bf8 ah, al;
          split_bf16(af[i], ah, al);
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
  }

#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (lb0 + i > lb_last) break;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = (cb0 + j) * 16 + r16;
      if (c >= ncol) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (lb0 + i) * 16 + 4 * g + v;
        if (row < a.nl) {
          const int64_t o = a.dtrans ? (int64_t)c * a.nl + row : (int64_t)row * ncol + c;
          a.delta[dbase + o] = acc[i][j][v];
        }
      }
    }
  }
}

template <int PREC, int MB, int NC>
hipError_t launch_t(const GemmArgs &a, int kcount, int max_ncol, hipStream_t s) {
  dim3 grid((unsigned)((a.nlb + 4 * MB - 1) / (4 * MB)),
            (unsigned)((max_ncol + 16 * NC - 1) / (16 * NC)), (unsigned)kcount);
  hipLaunchKernelGGL((mfma_gemm_kernel<PREC, MB, NC>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_p(const GemmArgs &a, const GemmTile &t, int kcount, int max_ncol,
                    hipStream_t s) {
  switch (t.mb * 16 + t.nc) {
    case 1 * 16 + 1: return launch_t<PREC, 1, 1>(a, kcount, max_ncol, s);
    case 2 * 16 + 1: return launch_t<PREC, 2, 1>(a, kcount, max_ncol, s);
    case 4 * 16 + 1: return launch_t<PREC, 4, 1>(a, kcount, max_ncol, s);
    case 2 * 16 + 2: return launch_t<PREC, 2, 2>(a, kcount, max_ncol, s);
    case 2 * 16 + 4: return launch_t<PREC, 2, 4>(a, kcount, max_ncol, s);
    case 4 * 16 + 2: return launch_t<PREC, 4, 2>(a, kcount, max_ncol, s);
    case 4 * 16 + 4: return launch_t<PREC, 4, 4>(a, kcount, max_ncol, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

GemmTile gemm_tile_at(int i) {
  static const GemmTile tiles[kGemmTileCount] = {{1, 1}, {2, 1}, {4, 1}, {2, 2},
                                                 {2, 4}, {4, 2}, {4, 4}, kGemmTileLds};
  return tiles[i];
}

bool gemm_tile_supported(const GemmTile &t) {
  if (t.mb == kGemmTileLds.mb && t.nc == kGemmTileLds.nc) return true;
  switch (t.mb * 16 + t.nc) {
    case 1 * 16 + 1: case 2 * 16 + 1: case 4 * 16 + 1: case 2 * 16 + 2:
    case 2 * 16 + 4: case 4 * 16 + 2: case 4 * 16 + 4:
      return true;
    default:
      return false;
  }
}

hipError_t mfma_gemm_launch(const GemmArgs &a, int prec, const GemmTile &t, int kcount,
                            int max_ncol, hipStream_t s) {
  if (t.mb == kGemmTileLds.mb && t.nc == kGemmTileLds.nc) {
    if (prec != 2) return hipErrorInvalidValue;  // the staged kernel is split-BF16x3 only
    return mfma_gemm_lds_launch(a, kcount, max_ncol, s);
  }
  if (prec == 1) return launch_p<1>(a, t, kcount, max_ncol, s);
  return launch_p<2>(a, t, kcount, max_ncol, s);
}

}  // namespace los
