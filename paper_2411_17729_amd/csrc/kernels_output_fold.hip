// Output pass with the last stages folded in (BF16 operands, padded m of 128
// and 256, q <= 16, p <= 64).
//
// The last s factors of eq. (2.2), stages k0 .. k0 + s - 1 with P_k = Abar^(2^k),
// multiply out to
//   prod_t (I + z^{-2^(k0+t)} P_{k0+t}) = sum_{j < 2^s} z^{-j 2^k0} Abar^(j 2^k0)
// (every j < 2^s once, by its binary digits). With G_j = C Abar^(j 2^k0), q x m,
// formed in FP64 during prepare, the output of the last display of §3 is
//   y_l = sum_{j < 2^s} G_j x_{l - j 2^k0} + D u_l,
// x the state after the stages before k0 (rows before the start zero). In the
// column numbering of stage k0 (block i of column c holds rows i 2^k0 + 16 c + r)
// the lags are the blocks i - j of the same column. A wave walks one column:
// block i of x adds G_j x_i to the outputs of block i + j, kept as 2^s + 3
// accumulators, and block i's y is complete once x_i itself is in. The G_j sit
// in LDS as MFMA A operands, staged once per workgroup; the waves exchange
// nothing else and meet at no barrier after that. x is loaded four blocks ahead
// and rounded to BF16 as the B operand, as every stage rounds its operands.
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

// S: folded stages (2^S lags); XB: the state is BF16
template <int MP, int S, bool XB>
__global__ __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_output_fold(
    StageParams prm, const FoldUnit* units) {
  constexpr int KS = MP / 32;        // MFMA steps of one contraction (32 entries each)
  constexpr int NL = 1 << S;         // lags
  constexpr int U = 4;               // blocks loaded ahead, and per unrolled group
  constexpr int NA = NL + U - 1;     // output blocks with partial sums
  constexpr int ES = XB ? 2 : 4;     // bytes of a state entry
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_fold[];
  bf16x8* gs = reinterpret_cast<bf16x8*>(smem_fold);                        // [NL][KS][64]
  float* ds = reinterpret_cast<float*>(smem_fold + (size_t)NL * KS * 64 * 16);  // D, q x p

  const FoldUnit un = units[blockIdx.x];
  const SeqDev sq = prm.seqs[un.seq];
  const OpDev o = prm.ops[sq.op];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int L = (int)sq.L, p = sq.p, q = sq.q;
  const int k0 = o.fold_k0;

  // G_j, packed in operand order (chunk (j, t, lane) holds G_j[lane % 16][32 t +
  // 8 (lane / 16) .. + 7]), and D into LDS; eight chunks per thread in flight
  {
    const bf16x8* gsrc = reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(prm.P) + o.fold_gc);
    constexpr int NC = NL * KS * 64;
    for (int e0 = 0; e0 < NC; e0 += 8 * 256) {
      bf16x8 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 256 * i + threadIdx.x;
        v[i] = e < NC ? gsrc[e] : bf16x8{};
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 256 * i + threadIdx.x;
        if (e < NC) gs[e] = v[i];
      }
    }
    const float* dm = reinterpret_cast<const float*>(prm.small) + o.dmat;
    for (int e = threadIdx.x; e < q * p; e += 256) ds[e] = dm[e];
    __syncthreads();
  }
  if (wave >= un.ncol) return;  // (no barrier follows)
  const int c = un.col0 + wave;
  const int ni = (L - 16 * c + (1 << k0) - 1) >> k0;  // blocks of this column with rows below L

  // x rows through a buffer resource over the sequence's L x MP block (rows
  // past L read as zero); y rows likewise (stores past L dropped)
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(reinterpret_cast<const unsigned char*>(prm.xin)) + sq.x_off * ES, (short)0,
      (int)nrec, kBufferWord3);
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float*>(prm.dst) + sq.y_off, (short)0,
                                                    (int)((uint32_t)L * (uint32_t)q * 4u), kBufferWord3);
  // this lane's piece of step t of a block: row r, entries 32 t + 8 g .. + 7
  const uint32_t lane_off = (uint32_t)(r * MP + 8 * g) * (uint32_t)ES;
  auto block_off = [&](int i) -> uint32_t {
    return i < ni ? lane_off + (uint32_t)((i << k0) + 16 * c) * (uint32_t)(MP * ES) : 0x80000000u;
  };
  f32x4 xr[U][KS][2];  // FP32 state
  u32x4 xh[U][KS];     // BF16 state
  auto issue = [&](int u, int i) {
    const uint32_t off = block_off(i);
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      if constexpr (XB) {
        xh[u][t] = __builtin_amdgcn_raw_buffer_load_b128(rin, off + 64 * t, 0, 0);
      } else {
        xr[u][t][0] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off + 128 * t, 0, 0));
        xr[u][t][1] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off + 128 * t + 16, 0, 0));
      }
    }
  };
#pragma unroll
  for (int u = 0; u < U; ++u) issue(u, u);

  // D u_l for this lane's row and outputs 4 g .. + 3 (inputs one row per lane)
  const bool vec = (p & 3) == 0 && src4_aligned(prm.src, prm.src_dtype, sq.u_off);
  auto du = [&](int l) -> f32x4 {
    f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t ub = sq.u_off + (int64_t)(l < L ? l : 0) * p;
    for (int cc = 0; cc < p; cc += 4) {
      f32x4 uv;
      if (vec) {
        uv = load_src4(prm.src, prm.src_dtype, ub + cc, true);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) uv[e] = cc + e < p ? load_src<float>(prm.src, prm.src_dtype, ub + cc + e) : 0.f;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int oo = 4 * g + v < q ? 4 * g + v : 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) d[v] += (cc + e < p ? ds[oo * p + cc + e] : 0.f) * uv[e];
      }
    }
    return d;
  };

  f32x4 acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < ni; i0 += U) {
    // the G_j operands are read from LDS at every block: an offset the
    // compiler cannot see through keeps it from hoisting them all into
    // registers (NL KS 4 VGPRs)
    int gz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(gz));
    const bf16x8* gsv = gs + gz;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      // block i as B operands (BF16, rounded to nearest even from FP32 state)
      bf16x8 b[KS];
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        if constexpr (XB) {
          b[t] = __builtin_bit_cast(bf16x8, xh[u][t]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            b[t][e] = (__bf16)xr[u][t][0][e];
            b[t][4 + e] = (__bf16)xr[u][t][1][e];
          }
        }
      }
      issue(u, i + U);
      // G_j x_i into the partial outputs of block i + j (lags past the
      // column's end go to blocks that are never stored)
#pragma unroll
      for (int j = 0; j < NL; ++j)
#pragma unroll
        for (int t = 0; t < KS; ++t)
          acc[u + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gsv[(j * KS + t) * 64 + lane], b[t], acc[u + j], 0, 0, 0);
      // block i is complete: y = its sums + D u (outputs 4 g + v of row r)
      const int l = (i << k0) + 16 * c + r;
      const f32x4 y = acc[u] + du(l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int oo = 4 * g + v;
        const uint32_t yoff = i < ni && l < L && oo < q ? (uint32_t)(l * q + oo) * 4u : 0x80000000u;
        const float yv = y[v];  // (a bit cast of the element itself reads element 0)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, yv), ry, yoff, 0, 0);
      }
    }
    // the group's U blocks are done: shift the partial sums down by U
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = a + U < NA ? acc[a + U] : f32x4{0.f, 0.f, 0.f, 0.f};
  }
}

template <int MP, int S, bool XB>
static hipError_t launch_fold_t(const StageParams& prm, const FoldUnit* units, int n_units, size_t lds,
                                hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_output_fold<MP, S, XB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_output_fold<MP, S, XB>), dim3(n_units), dim3(256), lds, s, prm, units);
  return hipGetLastError();
}

template <int MP, int S>
static hipError_t launch_fold_x(bool xb, const StageParams& prm, const FoldUnit* units, int n_units,
                                size_t lds, hipStream_t s) {
  return xb ? launch_fold_t<MP, S, true>(prm, units, n_units, lds, s)
            : launch_fold_t<MP, S, false>(prm, units, n_units, lds, s);
}

int fold_max_stages(int mp) { return mp == 256 ? 4 : mp == 128 ? 5 : 0; }

bool fold_supported(int mp, int ct, int s) {
  return ct == DT_BF16 && (mp == 128 || mp == 256) && s >= 2 && s <= fold_max_stages(mp);
}

size_t fold_lds(int mp, int s, int p, int q) {
  // G_j, then D (and four floats of slack for the grouped reads of its rows)
  return (size_t)(1 << s) * (mp / 32) * 64 * 16 + ((size_t)q * p + 4) * sizeof(float);
}

hipError_t launch_output_fold(int mp, int ct, int s, bool xb, const StageParams& prm, const FoldUnit* units,
                              int n_units, size_t lds, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  if (!fold_supported(mp, ct, s) || prm.adjoint || lds > 160 * 1024) return hipErrorInvalidValue;
  if (mp == 256) {
    switch (s) {
      case 2: return launch_fold_x<256, 2>(xb, prm, units, n_units, lds, st);
      case 3: return launch_fold_x<256, 3>(xb, prm, units, n_units, lds, st);
      case 4: return launch_fold_x<256, 4>(xb, prm, units, n_units, lds, st);
    }
  } else {
    switch (s) {
      case 2: return launch_fold_x<128, 2>(xb, prm, units, n_units, lds, st);
      case 3: return launch_fold_x<128, 3>(xb, prm, units, n_units, lds, st);
      case 4: return launch_fold_x<128, 4>(xb, prm, units, n_units, lds, st);
      case 5: return launch_fold_x<128, 5>(xb, prm, units, n_units, lds, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ssmc
