// Shared pieces of the stage kernels that keep the power resident in LDS.
#pragma once
#include "stage_common.h"

namespace ssmc {

template <int MP, int CT>
struct ResCfg {
  using TR = CTraits<CT>;
  using X = typename TR::X;
  using Op = typename TR::Op;
  static constexpr int NS = (size_t)MP * MP * sizeof(Op) > 136 * 1024 ? 2 : 1;
  static constexpr int NR = MP / NS;  // output state rows per workgroup
  static constexpr int NB = NR / 16;  // 16-row output blocks per wave
  static constexpr int PADP = 16 / (int)sizeof(Op);
  static constexpr int SP = MP + PADP;  // LDS row stride (elements)
  static constexpr int WAVES = 8;
  static constexpr size_t LDS = (size_t)NR * SP * sizeof(Op);
  static constexpr int NV = MP / 16;  // float4 pieces of a shifted row held per lane
};

// Output epilogue on the matrix cores: for the lane's 16-row block,
//     Y^T[qq, l] = sum_n Cm[qq, n] X^T[n, l] + sum_c Dm[qq, c] V^T[c, l]
// (y = C x + D u forward, du = Bbar^T g + D^T dy adjoint), 16 outputs at a
// time with the FP32 16x16x4 MFMA. The state block is used where it lies:
// accumulator entry v of block nb (state index 16 nb + 4 g + v, time row j)
// is the B operand of step (nb, v), whose contraction index 4-group is g, so
// the A operand of lane (i, g) is Cm[q0 + i][16 nb + 4 g + v]. The inputs V
// enter the same accumulator, four channels per step. The result lane (j, g)
// holds outputs q0 + 4 g + v of time row l.
template <int NB>
__device__ __forceinline__ void res_epilogue(const f32x4 (&acc)[NB], int mp, int64_t l, bool lv,
                                             const float* cm, const float* dm, int w, int r_in,
                                             const void* src, int sdt, int64_t src_off,
                                             float* dst, int64_t dst_off, int j, int g) {
  for (int q0 = 0; q0 < w; q0 += 16) {
    const int qi = q0 + j;
    const bool qv = qi < w;
    f32x4 ya = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const f32x4 cv = qv ? *reinterpret_cast<const f32x4*>(cm + (int64_t)qi * mp + nb * 16 + 4 * g)
                          : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) ya = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[v], acc[nb][v], ya, 0, 0, 0);
    }
    for (int a = 0; a < (r_in + 3) / 4; ++a) {
      const int c = 4 * a + g;
      const float dv = qv && c < r_in ? dm[qi * r_in + c] : 0.f;
      const float uv = lv && c < r_in ? load_src<float>(src, sdt, src_off + l * r_in + c) : 0.f;
      ya = __builtin_amdgcn_mfma_f32_16x16x4f32(dv, uv, ya, 0, 0, 0);
    }
    if (lv) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int qq = q0 + 4 * g + v;
        if (qq < w) dst[dst_off + l * w + qq] = ya[v];
      }
    }
  }
}

}  // namespace ssmc
