// Output of a sequence's last stage, for stage launches that ran without
// their epilogue: FP32 at padded m 256, where a stage's output rows are split
// between two workgroups and neither holds a whole row (the output of the
// last display of §3 needs all of x_l):
//   forward:  y_l  = C x_l + D u_l
//   adjoint:  du_l = Bbar^T g_l + D^T dy_l
// from the state rows the stage stored. One workgroup of four waves per
// range of rows of one sequence; a wave takes 16-row blocks. The rows of C
// (or Bbar^T) are MFMA A operands in registers, the state rows B operands in
// the layout of the stage kernels' accumulators (lane (row j, group g) holds
// entries 16 a + 4 g .. 16 a + 4 g + 3 of its row), so FP32 step (a, t)
// contracts entry 16 a + 4 g + t; lane (j, g) ends with outputs 4 g .. 4 g + 3
// of row j, to which it adds D u_l on the vector units.
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

template <int MP>
__global__ __launch_bounds__(256) void k_output_proj(StageParams prm, const ResRange* ranges) {
  constexpr int NV = MP / 16;
  const ResRange rg = ranges[blockIdx.x];
  const SeqDev sq = prm.seqs[rg.seq];
  const bool adj = prm.adjoint != 0;
  const int k = prm.k;
  // the stage launch's own tests: only where this is the sequence's last
  // stage of the direction and the stage ran for it
  if (k > sq.last) return;
  if (prm.skip_kry && k < sq.kry) return;
  if (adj ? k != 0 : k != sq.last) return;
  const OpDev o = prm.ops[sq.op];
  const float* cm = reinterpret_cast<const float*>(prm.small) + (adj ? o.bt : o.cout);  // ew x MP
  const float* dm = reinterpret_cast<const float*>(prm.small) + (adj ? o.dt : o.dmat);  // ew x er
  const int ew = adj ? sq.p : sq.q, er = adj ? sq.q : sq.p;
  const int64_t so = adj ? sq.y_off : sq.u_off, dof = adj ? sq.u_off : sq.y_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  __shared__ float ds[16 * 16];  // D (or D^T), ew x er
  for (int e = threadIdx.x; e < ew * er; e += 256) ds[e] = dm[e];
  __syncthreads();

  f32x4 ca[NV];  // row j of C (zero past ew), entries 16 a + 4 g ..
#pragma unroll
  for (int a = 0; a < NV; ++a)
    ca[a] = j < ew ? *reinterpret_cast<const f32x4*>(cm + (int64_t)j * MP + 16 * a + 4 * g)
                   : f32x4{0.f, 0.f, 0.f, 0.f};

  // the sequence's rows through a buffer resource: rows at or past L read zero
  const int L = (int)sq.L;
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * sizeof(float));
  const auto rx = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float*>(prm.xout) + sq.x_off, (short)0,
                                                    (int)nrec, kBufferWord3);
  float* dst = reinterpret_cast<float*>(prm.dst);
  const int nblk = (rg.nrows + 15) >> 4;
  for (int b = wave; b < nblk; b += 4) {
    const int l = rg.row0 + 16 * b + j;
    const uint32_t off = (uint32_t)l * (uint32_t)(MP * sizeof(float)) + 16u * (uint32_t)g;
    f32x4 xv[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a)
      xv[a] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rx, off + 64u * a, 0, 0));
    // the row's inputs, loaded before the contraction so that they arrive
    // during it
    const bool live = l < L && l < rg.row0 + rg.nrows;
    float uv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c)
      uv[c] = live && c < er ? load_src<float>(prm.src, prm.src_dtype, so + (int64_t)l * er + c) : 0.f;
    // four accumulator chains (steps t), added at the end
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[a][t], xv[a][t], acc[t], 0, 0, 0);
    if (live) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int out = 4 * g + v;
        if (out < ew) {
          float yv = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
#pragma unroll
          for (int c = 0; c < 16; ++c)
            if (c < er) yv = fmaf(ds[out * er + c], uv[c], yv);
          dst[dof + (int64_t)l * ew + out] = yv;
        }
      }
    }
  }
}

bool output_proj_supported(int mp, int ct, int ew, int er) {
  return ct == DT_F32 && mp == 256 && ew >= 1 && ew <= 16 && er >= 0 && er <= 16;
}

hipError_t launch_output_proj(int mp, const StageParams& prm, const ResRange* ranges, int n_ranges,
                              hipStream_t s) {
  if (n_ranges <= 0) return hipSuccess;
  if (mp != 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_output_proj<256>), dim3(n_ranges), dim3(256), 0, s, prm, ranges);
  return hipGetLastError();
}

}  // namespace ssmc
