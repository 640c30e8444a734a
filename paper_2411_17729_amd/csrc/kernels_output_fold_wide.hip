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
// (the top rows to one, the bottom rows to the next). In the column numbering
// of stage k0 (block i of column c holds rows i 2^k0 + 16 c + r) a workgroup
// walks one column in groups of four blocks. Its eight waves split the lags,
// wave w holding the operands of lags 8 w .. 8 w + 7 in registers; the group's
// blocks are loaded two groups ahead by all 512 threads, rounded to BF16 (the
// operand type) and staged in LDS in operand order, so every wave reads a B
// operand with one 16-byte read and the state is read from HBM once. Output
// block o collects the waves' partial sums in an LDS ring slot, in a fixed
// order: wave w finishes its part of o in the group that holds block o - 8 w,
// so the last wave adds first and the first wave, which finishes o last, adds
// its part to the slot and stores y; D u is added by the last wave a group
// ahead. Within a wave, the partial sums of output block o sit in the top rows
// of one accumulator and the bottom rows of the one before, and are joined
// with one cross-lane exchange.
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

namespace {
constexpr int kWideMp = 256;
constexpr int kWideKs = kWideMp / 32;  // MFMA steps of one contraction
constexpr int kWideNw = 8;             // waves: lags 8 w .. 8 w + 7 each
constexpr int kWideU = 2;              // blocks per group
constexpr int kWideRing = 64 + kWideU; // output slots in flight
constexpr size_t kWideXs = (size_t)2 * kWideU * kWideKs * 64 * 16;  // two groups of operand blocks
constexpr size_t kWideLds = kWideXs + (size_t)kWideRing * 32 * 16;
}  // namespace

template <bool XB>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_output_fold_wide(
    StageParams prm, const FoldUnit* units) {
  constexpr int MP = kWideMp, KS = kWideKs, NW = kWideNw, U = kWideU, R = kWideRing;
  constexpr int NPW = 4;             // paired operands of a wave (8 lags)
  constexpr int NA = U + 2 * NPW;    // accumulators, offsets -1 .. U + 2 NPW - 2
  constexpr int ES = XB ? 2 : 4;     // bytes of a state entry
  constexpr int PM = 2;              // FP32 MFMA steps of D u loaded ahead (p <= 8)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_foldw[];
  bf16x8* xs = reinterpret_cast<bf16x8*>(smem_foldw);                 // [2][U][KS][64]
  f32x4* outs = reinterpret_cast<f32x4*>(smem_foldw + kWideXs);       // [R][32]

  const FoldUnit un = units[blockIdx.x];
  const SeqDev sq = prm.seqs[un.seq];
  const OpDev o = prm.ops[sq.op];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int L = (int)sq.L, p = sq.p, q = sq.q;
  const int k0 = o.fold_k0;
  const int c = un.col0;
  const int no = (L - 16 * c + (1 << k0) - 1) >> k0;  // blocks of the column with rows below L

  // this wave's paired operands (lags 8 wave .. + 7) in registers
  bf16x8 ga[NPW][KS];
  {
    const bf16x8* gsrc = reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(prm.P) + o.fold_gc);
#pragma unroll
    for (int i = 0; i < NPW; ++i)
#pragma unroll
      for (int t = 0; t < KS; ++t) ga[i][t] = gsrc[((NPW * wave + i) * KS + t) * 64 + lane];
  }
  for (int e = threadIdx.x; e < R * 32; e += 512) outs[e] = f32x4{0.f, 0.f, 0.f, 0.f};

  // staging: thread s holds operand chunk s of a block (step t = s / 64,
  // lane s % 64): row s % 16, entries 32 t + 8 ((s / 16) % 4) .. + 7. A wave
  // writes 64 consecutive chunks, and the four lanes of a row read 64 (BF16)
  // or 128 (FP32) contiguous bytes
  const int sr = threadIdx.x & 15, c8 = ((threadIdx.x >> 6) << 2) | ((threadIdx.x >> 4) & 3);
  const uint32_t soff = (uint32_t)(sr * MP + 8 * c8) * (uint32_t)ES;
  const int schunk = threadIdx.x;
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(reinterpret_cast<const unsigned char*>(prm.xin)) + sq.x_off * ES, (short)0,
      (int)nrec, kBufferWord3);
  auto boff = [&](int i) -> uint32_t {
    return i < no ? soff + (uint32_t)((i << k0) + 16 * c) * (uint32_t)(MP * ES) : 0x80000000u;
  };
  f32x4 stf[2][U][2];  // FP32 state: two groups in flight
  u32x4 sth[2][U];     // BF16 state
  auto load_group = [&](int set, int gi) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t off = boff(gi * U + u);
      if constexpr (XB) {
        sth[set][u] = __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0);
      } else {
        stf[set][u][0] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0));
        stf[set][u][1] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off + 16, 0, 0));
      }
    }
  };
  auto write_group = [&](int set, int buf) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bf16x8 v;
      if constexpr (XB) {
        v = __builtin_bit_cast(bf16x8, sth[set][u]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e] = (__bf16)stf[set][u][0][e];  // round to nearest even
          v[4 + e] = (__bf16)stf[set][u][1][e];
        }
      }
      xs[(buf * U + u) * KS * 64 + schunk] = v;
    }
  };

  // D u of the next group's outputs, formed by the last wave (the least work)
  // and added into their ring slots a group before the first wave takes them
  const bool du_wave = wave == NW - 1;
  const bool ubf = prm.src_dtype != DT_F32;
  const unsigned char* ub = reinterpret_cast<const unsigned char*>(prm.src) + sq.u_off * (ubf ? 2 : 4);
  const uint32_t ulead = (uint32_t)(reinterpret_cast<uintptr_t>(ub) & 3);
  const auto ru = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(ub - ulead), (short)0,
                                                    (int)((ulead + (uint32_t)L * (uint32_t)p * (ubf ? 2u : 4u) + 3u) & ~3u),
                                                    kBufferWord3);
  const int pm = (p + 3) / 4;
  const uint32_t ush = ubf ? 1u : 2u, urow = (uint32_t)(16 * c + r);
  auto u_byte = [&](int i, int m) -> uint32_t {
    const uint32_t e = (((uint32_t)i << k0) + urow) * (uint32_t)p + (uint32_t)(4 * m + g);
    return (e << ush) + ulead;
  };
  auto u_word = [&](int i, int m) {
    const bool ok = (i < no) & ((((uint32_t)i << k0) + urow) < (uint32_t)L) & (4 * m + g < p);
    return __builtin_amdgcn_raw_buffer_load_b32(ru, ok ? u_byte(i, m) & ~3u : 0x80000000u, 0, 0);
  };
  auto u_val = [&](uint32_t w, int i, int m) {
    const uint32_t sh = ubf && !(u_byte(i, m) & 2u) ? 16u : 0u;
    return __uint_as_float((w << sh) & (ubf ? 0xffff0000u : 0xffffffffu));
  };
  const float* dm = reinterpret_cast<const float*>(prm.small) + o.dmat;
  auto d_at = [&](int m) { return r < q && 4 * m + g < p ? dm[r * p + 4 * m + g] : 0.f; };
  float da[PM];
  uint32_t uw[U][PM];
  auto u_issue = [&](int gi) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < PM; ++m) uw[u][m] = u_word(gi * U + u, m);
  };
  // D u of group gi's blocks into their slots (lanes of rows 0 .. 7)
  auto du_add = [&](int gi) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ob = gi * U + u;
      f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < PM; ++m) d = __builtin_amdgcn_mfma_f32_16x16x4f32(da[m], u_val(uw[u][m], ob, m), d, 0, 0, 0);
      for (int m = PM; m < pm; ++m) d = __builtin_amdgcn_mfma_f32_16x16x4f32(d_at(m), u_val(u_word(ob, m), ob, m), d, 0, 0, 0);
      if (g < 2 && ob < no) {
        f32x4* sl = outs + (ob % R) * 32 + lane;
        *sl = *sl + d;
      }
    }
  };

  load_group(0, 0);
  load_group(1, 1);
  if (du_wave) {
#pragma unroll
    for (int m = 0; m < PM; ++m) da[m] = d_at(m);
    u_issue(0);
  }
  write_group(0, 0);
  load_group(0, 2);
  __syncthreads();  // the ring is zero, group 0 staged
  if (du_wave) {
    du_add(0);
    u_issue(1);
  }
  __syncthreads();  // D u of group 0 in its slots before the first wave takes them

  f32x4 acc[NA];  // acc[a]: output offset a - 1 (top rows), a (bottom rows), from i0 + 8 wave
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool y4 = (q & 3) == 0 && (reinterpret_cast<uintptr_t>(reinterpret_cast<float*>(prm.dst) + sq.y_off) & 15) == 0;
  float* ydst = reinterpret_cast<float*>(prm.dst) + sq.y_off;
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(ydst, (short)0, (int)((uint32_t)L * (uint32_t)q * 4u), kBufferWord3);
  // one group; SET (= (gi + 1) % 2) is a constant so the register sets of
  // the loads in flight are never indexed at run time
  auto group = [&](int gi, auto set_c) {
    constexpr int SET = decltype(set_c)::value;
    const int i0 = gi * U, buf = SET ^ 1;
    if (i0 + 8 * wave < no) {
      // block i0 + u through operand i into accumulator u + 2 i + 1
#pragma unroll
      for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bf16x8 b = xs[((buf * U + u) * KS + t) * 64 + lane];
#pragma unroll
          for (int i = 0; i < NPW; ++i)
            acc[u + 2 * i + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ga[i][t], b, acc[u + 2 * i + 1], 0, 0, 0);
        }
    }
    // outputs i0 + 8 wave + u are complete for this wave's lags: top rows of
    // accumulator u + 1 and bottom rows (lanes 32 .. 63) of accumulator u;
    // the first wave finishes them into y, the others add into their slots
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ob = i0 + 8 * wave + u;
      f32x4 val;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float lo = acc[u][v];
        val[v] = acc[u + 1][v] + __shfl_xor(lo, 32);
      }
      if (g < 2 && ob < no) {
        f32x4* sl = outs + (ob % R) * 32 + lane;
        if (wave != 0) {
          *sl = *sl + val;
        } else {
          const f32x4 y = *sl + val;
          *sl = f32x4{0.f, 0.f, 0.f, 0.f};
          const int l = (ob << k0) + 16 * c + r;
          if (y4) {
            const uint32_t yoff = l < L && 4 * g < q ? (uint32_t)(l * q + 4 * g) * 4u : 0x80000000u;
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, y), ry, yoff, 0, 0);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int oo = 4 * g + v;
              const uint32_t yoff = l < L && oo < q ? (uint32_t)(l * q + oo) * 4u : 0x80000000u;
              const float yv = y[v];  // (a bit cast of the element itself reads element 0)
              __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, yv), ry, yoff, 0, 0);
            }
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = a + U < NA ? acc[a + U] : f32x4{0.f, 0.f, 0.f, 0.f};
    if (du_wave) {
      du_add(gi + 1);
      u_issue(gi + 2);
    }
    // group gi + 1 into the other operand buffer, group gi + 3 into its registers
    write_group(SET, SET);
    load_group(SET, gi + 3);
    __syncthreads();
  };
  for (int gi = 0; gi * U < no; gi += 2) {
    group(gi, std::integral_constant<int, 1>{});
    if ((gi + 1) * U >= no) break;
    group(gi + 1, std::integral_constant<int, 0>{});
  }
}

template <bool XB>
static hipError_t launch_wide_t(const StageParams& prm, const FoldUnit* units, int n_units, hipStream_t s) {
  {
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_output_fold_wide<XB>), (size_t)(160 * 1024));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_output_fold_wide<XB>), dim3(n_units), dim3(512), fold_wide_lds(), s, prm, units);
  return hipGetLastError();
}

bool fold_wide_supported(int mp, int ct, int q, int p) {
  return ct == DT_BF16 && mp == kWideMp && q >= 1 && q <= 8 && p >= 1 && p <= 64;
}

size_t fold_wide_lds() { return kWideLds; }

hipError_t launch_output_fold_wide(int mp, int ct, bool xb, const StageParams& prm, const FoldUnit* units,
                                   int n_units, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  if (mp != kWideMp || ct != DT_BF16 || prm.adjoint) return hipErrorInvalidValue;
  return xb ? launch_wide_t<true>(prm, units, n_units, st) : launch_wide_t<false>(prm, units, n_units, st);
}

}  // namespace ssmc
