// Output pass with six stages folded in, for q <= 8 at padded m = 256 (BF16
// operands).
//
// As in the narrower output fold, the last s factors of eq. (2.2) multiply out
// to sum_{j < 2^s} z^{-j 2^k0} Abar^(j 2^k0), so with G_j = C Abar^(j 2^k0)
// (q x m, formed in FP64 during prepare) the output of the last display of §3
// is
//   y_l = sum_{j < 64} G_j x_{l - j 2^k0} + D u_l,
// x the state after the stages before k0. With q <= 8, two lags share one
// MFMA A operand: rows 0..7 hold G_{2i}, rows 8..15 G_{2i+1}, so one 16 x 16 x
// 32 product of a state block gives its contributions to two output blocks
// (the top rows to block i + 2i', the bottom rows to the one after). This
// halves the products and the LDS the G_j take: 32 lags fill 128 KB. The 64
// lags are split in two ranges of 32, each handled by its own workgroups
// (the field jlo of the unit: 0 or 32), and both add their partial outputs
// into y, which a fill kernel has zeroed first: every output gets at most two
// additions onto zero, so the result does not depend on their order. The
// range from 32 reads only the state blocks that still have outputs 32 or
// more blocks later. In the column numbering of stage k0 (block i of column c
// holds rows i 2^k0 + 16 c + r) a wave walks one column in groups of U blocks
// as the narrower fold does; the partial sums of output block o sit in the
// top rows of accumulator o and the bottom rows of accumulator o - 1, and are
// joined with one cross-lane exchange when the block is complete.
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

namespace {
constexpr int kWideMp = 256;
constexpr int kWideNp = 16;  // paired A operands of a range (32 lags)
}  // namespace

template <bool XB>
__global__ __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_output_fold_wide(
    StageParams prm, const FoldUnit* units) {
  constexpr int MP = kWideMp;
  constexpr int KS = MP / 32;     // MFMA steps of one contraction
  constexpr int NP = kWideNp;     // paired operands (lags 2 i', 2 i' + 1 of the range)
  constexpr int U = XB ? 4 : 3;   // blocks per group, loaded a group ahead
  constexpr int NA = U + 2 * NP - 1;  // accumulators, output offsets -1 .. U + 2 NP - 3
  constexpr int ES = XB ? 2 : 4;  // bytes of a state entry
  constexpr int PM = 2;           // FP32 MFMA steps of D u loaded ahead (p <= 8)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_foldw[];
  bf16x8* gs = reinterpret_cast<bf16x8*>(smem_foldw);  // [NP][KS][64]

  const FoldUnit un = units[blockIdx.x];
  const SeqDev sq = prm.seqs[un.seq];
  const OpDev o = prm.ops[sq.op];
  const int jlo = un.reserved;  // first lag of the range: 0 or 2 NP
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int L = (int)sq.L, p = sq.p, q = sq.q;
  const int k0 = o.fold_k0;
  const bool active = wave < un.ncol;
  const bool with_du = jlo == 0;  // the first range adds D u
  const int c = un.col0 + wave;
  // output blocks of this column with rows below L, and the input blocks with
  // an output in the range (i + jlo < no)
  const int no = active ? (L - 16 * c + (1 << k0) - 1) >> k0 : 0;
  const int ni = no > jlo ? no - jlo : 0;

  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(reinterpret_cast<const unsigned char*>(prm.xin)) + sq.x_off * ES, (short)0,
      (int)nrec, kBufferWord3);
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float*>(prm.dst) + sq.y_off, (short)0,
                                                    (int)((uint32_t)L * (uint32_t)q * 4u), kBufferWord3);
  // u through one 4-byte load per input for either type (BF16 inputs from the
  // aligned word that holds them)
  const bool ubf = prm.src_dtype != DT_F32;
  const unsigned char* ub = reinterpret_cast<const unsigned char*>(prm.src) + sq.u_off * (ubf ? 2 : 4);
  const uint32_t ulead = (uint32_t)(reinterpret_cast<uintptr_t>(ub) & 3);
  const auto ru = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(ub - ulead), (short)0,
                                                    (int)((ulead + (uint32_t)L * (uint32_t)p * (ubf ? 2u : 4u) + 3u) & ~3u),
                                                    kBufferWord3);
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
  // D u on FP32 MFMA, as in the narrower fold (output block i of the first
  // range is input block i)
  const int pm = (p + 3) / 4;
  const uint32_t ush = ubf ? 1u : 2u, urow = (uint32_t)(16 * c + r);
  auto u_byte = [&](int i, int m) -> uint32_t {
    const uint32_t e = (((uint32_t)i << k0) + urow) * (uint32_t)p + (uint32_t)(4 * m + g);
    return (e << ush) + ulead;
  };
  auto u_word = [&](int i, int m) {
    const bool ok = with_du & (i < no) & ((((uint32_t)i << k0) + urow) < (uint32_t)L) & (4 * m + g < p);
    return __builtin_amdgcn_raw_buffer_load_b32(ru, ok ? u_byte(i, m) & ~3u : 0x80000000u, 0, 0);
  };
  auto u_val = [&](uint32_t w, int i, int m) {
    const uint32_t sh = ubf && !(u_byte(i, m) & 2u) ? 16u : 0u;
    return __uint_as_float((w << sh) & (ubf ? 0xffff0000u : 0xffffffffu));
  };
  uint32_t uw[U][PM];
  auto u_issue = [&](int i0n) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < PM; ++m) uw[u][m] = u_word(i0n + u, m);
  };
  u_issue(0);
#pragma unroll
  for (int u = 0; u < U; ++u) issue(u, u);

  // the range's paired operands into LDS (chunk (i', t, lane) holds rows lane
  // % 16 of G_{jlo + 2 i'} over G_{jlo + 2 i' + 1}, entries 32 t + 8 (lane /
  // 16) .. + 7); eight chunks per thread in flight
  {
    const bf16x8* gsrc = reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(prm.P) + o.fold_gc) +
                         (size_t)(jlo / 2) * KS * 64;
    constexpr int NC = NP * KS * 64;
    for (int e0 = 0; e0 < NC; e0 += 8 * 256) {
      bf16x8 v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = gsrc[e0 + 256 * i + threadIdx.x];
#pragma unroll
      for (int i = 0; i < 8; ++i) gs[e0 + 256 * i + threadIdx.x] = v[i];
    }
    __syncthreads();
  }
  if (!active) return;  // (no barrier follows)

  const float* dm = reinterpret_cast<const float*>(prm.small) + o.dmat;
  auto d_at = [&](int m) { return with_du && r < q && 4 * m + g < p ? dm[r * p + 4 * m + g] : 0.f; };
  float da[PM];
#pragma unroll
  for (int m = 0; m < PM; ++m) da[m] = d_at(m);

  f32x4 acc[NA];  // acc[a]: output offset a - 1 (top rows), a (bottom rows)
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < ni; i0 += U) {
    int gz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(gz));
    const bf16x8* gsv = gs + gz;
    if (with_du) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int m = 0; m < PM; ++m)
          acc[u + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[m], u_val(uw[u][m], i0 + u, m), acc[u + 1], 0, 0, 0);
        for (int m = PM; m < pm; ++m)
          acc[u + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(d_at(m), u_val(u_word(i0 + u, m), i0 + u, m),
                                                            acc[u + 1], 0, 0, 0);
      }
    }
    bf16x8 b[U][KS];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        if constexpr (XB) {
          b[u][t] = __builtin_bit_cast(bf16x8, xh[u][t]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            b[u][t][e] = (__bf16)xr[u][t][0][e];
            b[u][t][4 + e] = (__bf16)xr[u][t][1][e];
          }
        }
      }
    u_issue(i0 + U);
#pragma unroll
    for (int u = 0; u < U; ++u) issue(u, i0 + U + u);
    // block i0 + u through operand i' into accumulator u + 2 i' + 1 (outputs
    // i0 + jlo + u + 2 i' and the one after); operands in pairs (four lags),
    // a pair skipped when every output it would reach lies past the column
#pragma unroll
    for (int jq = 0; jq < NP / 2; ++jq) {
      if (i0 + jlo + 4 * jq < no) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int jp = 2 * jq + jj;
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const bf16x8 a = gsv[(jp * KS + t) * 64 + lane];
#pragma unroll
            for (int u = 0; u < U; ++u)
              acc[u + 2 * jp + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[u][t], acc[u + 2 * jp + 1], 0, 0, 0);
          }
        }
        constexpr int NR = 2 * KS;  // reads of the two operands
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int k = 0; k < NR - 4; ++k) {
          __builtin_amdgcn_sched_group_barrier(0x008, U, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * U, 0);
      }
    }
    // outputs i0 + jlo + u are complete for this range: the top rows of
    // accumulator u + 1 and the bottom rows of accumulator u (lanes 32 .. 63
    // hold rows 8 .. 15), added into y (outputs 4 g + v of row r, g < 2)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ob = i0 + jlo + u;
      const int l = (ob << k0) + 16 * c + r;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float lo = acc[u][v];
        const float below = __shfl_xor(lo, 32);
        const float hi = acc[u + 1][v];
        const int oo = 4 * g + v;
        const uint32_t yoff = g < 2 && ob < no && l < L && oo < q ? (uint32_t)(l * q + oo) * 4u : 0x80000000u;
        __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(hi + below, ry, yoff, 0, 0);
      }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = a + U < NA ? acc[a + U] : f32x4{0.f, 0.f, 0.f, 0.f};
  }
}

// y of every sequence the units cover set to zero (one unit of each sequence
// has col0 = 0 and jlo = 0), before the ranges add into it
__global__ void k_fold_zero_y(StageParams prm, const FoldUnit* units) {
  const FoldUnit un = units[blockIdx.y];
  if (un.col0 != 0 || un.reserved != 0) return;
  const SeqDev sq = prm.seqs[un.seq];
  float* y = reinterpret_cast<float*>(prm.dst) + sq.y_off;
  const int64_t n = sq.L * (int64_t)sq.q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = 0.f;
}

template <bool XB>
static hipError_t launch_wide_t(const StageParams& prm, const FoldUnit* units, int n_units, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_output_fold_wide<XB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_output_fold_wide<XB>), dim3(n_units), dim3(256), fold_wide_lds(), s, prm, units);
  return hipGetLastError();
}

bool fold_wide_supported(int mp, int ct, int q, int p) {
  return ct == DT_BF16 && mp == kWideMp && q >= 1 && q <= 8 && p >= 1 && p <= 64;
}

size_t fold_wide_lds() { return (size_t)kWideNp * (kWideMp / 32) * 64 * 16; }

hipError_t launch_output_fold_wide(int mp, int ct, bool xb, const StageParams& prm, const FoldUnit* units,
                                   int n_units, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  if (mp != kWideMp || ct != DT_BF16 || prm.adjoint) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fold_zero_y, dim3(64, n_units), dim3(256), 0, st, prm, units);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return xb ? launch_wide_t<true>(prm, units, n_units, st) : launch_wide_t<false>(prm, units, n_units, st);
}

}  // namespace ssmc
