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
// the lags are the blocks i - j of the same column. A wave walks one column in
// groups of four blocks: block i of x adds G_j x_i to the outputs of block
// i + j, kept as 2^s + 3 accumulators, and a group's outputs are complete once
// its own blocks are in. Each step of G_j is read from LDS once per group and
// serves its four blocks; lags that only reach past the column's end are
// skipped four at a time. The G_j sit in LDS as MFMA A operands, staged once per
// workgroup; the waves exchange nothing else and meet at no barrier after
// that. x is loaded a group ahead and rounded to BF16 as the B operand, as
// every stage rounds its operands.
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

// S: folded stages (2^S lags); XB: the state is BF16
template <int MP, int S, bool XB>
__global__ __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_output_fold(
    StageParams prm, const FoldUnit* units) {
  constexpr int KS = MP / 32;  // MFMA steps of one contraction (32 entries each)
  constexpr int NL = 1 << S;   // lags
  // blocks per group, loaded a group ahead: 2 U KS 16-byte loads per lane of
  // FP32 state, U KS of BF16, kept with the rest of a group's loads and stores
  // under the 63 vector memory operations a wave can have outstanding
  constexpr int U = XB ? 4 : 3;
  constexpr int NA = NL + U - 1;  // output blocks with partial sums
  constexpr int ES = XB ? 2 : 4;  // bytes of a state entry
  constexpr int PM = 2;           // FP32 MFMA steps of D u loaded ahead (p <= 8)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_fold[];
  bf16x8* gs = reinterpret_cast<bf16x8*>(smem_fold);  // [NL][KS][64]

  const FoldUnit un = units[blockIdx.x];
  const SeqDev sq = prm.seqs[un.seq];
  const OpDev o = prm.ops[sq.op];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int L = (int)sq.L, p = sq.p, q = sq.q;
  const int k0 = o.fold_k0;
  const bool active = wave < un.ncol;
  const int c = un.col0 + wave;
  // blocks of this column with rows below L (none for a wave past the unit)
  const int ni = active ? (L - 16 * c + (1 << k0) - 1) >> k0 : 0;

  // x rows through a buffer resource over the sequence's L x MP block (rows
  // past L read as zero); u and y rows likewise (stores past L dropped)
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(reinterpret_cast<const unsigned char*>(prm.xin)) + sq.x_off * ES, (short)0,
      (int)nrec, kBufferWord3);
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float*>(prm.dst) + sq.y_off, (short)0,
                                                    (int)((uint32_t)L * (uint32_t)q * 4u), kBufferWord3);
  // u through one 4-byte load per input for either type: BF16 inputs are read
  // as the aligned word that holds them (never crossing past the word of the
  // block's last input) and taken from its low or high half
  const bool ubf = prm.src_dtype != DT_F32;
  const unsigned char* ub = reinterpret_cast<const unsigned char*>(prm.src) + sq.u_off * (ubf ? 2 : 4);
  const uint32_t ulead = (uint32_t)(reinterpret_cast<uintptr_t>(ub) & 3);  // 0 or 2 (BF16)
  const auto ru = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(ub - ulead), (short)0,
                                                    (int)((ulead + (uint32_t)L * (uint32_t)p * (ubf ? 2u : 4u) + 3u) & ~3u),
                                                    kBufferWord3);
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

  // D u on FP32 MFMA (16 x 16 x 4 per step m, inputs 4 m .. + 3): A = D[lane %
  // 16][4 m + lane / 16] (zero past q and p), B = u[row lane % 16][4 m + lane /
  // 16], one value per lane and step. The first PM steps have their A in
  // registers and their B loaded just before the group's x blocks, a group
  // ahead; steps past them (p > 4 PM) load both where they are used.
  const int pm = (p + 3) / 4;  // steps
  // byte offset of input 4 m + g of row i 2^k0 + 16 c + r from the aligned base
  // (branch-free: the loads stay where they are issued)
  const uint32_t ush = ubf ? 1u : 2u, urow = (uint32_t)(16 * c + r);
  auto u_byte = [&](int i, int m) -> uint32_t {
    const uint32_t e = (((uint32_t)i << k0) + urow) * (uint32_t)p + (uint32_t)(4 * m + g);
    return (e << ush) + ulead;
  };
  auto u_word = [&](int i, int m) {
    const bool ok = (i < ni) & ((((uint32_t)i << k0) + urow) < (uint32_t)L) & (4 * m + g < p);
    return __builtin_amdgcn_raw_buffer_load_b32(ru, ok ? u_byte(i, m) & ~3u : 0x80000000u, 0, 0);
  };
  // the input as FP32 from its word: BF16 from the low or high half
  auto u_val = [&](uint32_t w, int i, int m) {
    const uint32_t sh = ubf && !(u_byte(i, m) & 2u) ? 16u : 0u;
    return __uint_as_float((w << sh) & (ubf ? 0xffff0000u : 0xffffffffu));
  };
  // words of the inputs loaded ahead, widened where they are used
  uint32_t uw[U][PM];
  auto u_issue = [&](int i0n) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < PM; ++m) uw[u][m] = u_word(i0n + u, m);
  };
  // the first group's u and x loads go out before the G_j are staged
  u_issue(0);
#pragma unroll
  for (int u = 0; u < U; ++u) issue(u, u);

  // G_j, packed in operand order (chunk (j, t, lane) holds G_j[lane % 16][32 t +
  // 8 (lane / 16) .. + 7]), into LDS; eight chunks per thread in flight
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
    __syncthreads();
  }
  if (!active) return;  // (no barrier follows)

  const float* dm = reinterpret_cast<const float*>(prm.small) + o.dmat;
  auto d_at = [&](int m) { return r < q && 4 * m + g < p ? dm[r * p + 4 * m + g] : 0.f; };
  float da[PM];
#pragma unroll
  for (int m = 0; m < PM; ++m) da[m] = d_at(m);
  // y rows: the four outputs 4 g .. + 3 of a lane in one store where q is a
  // multiple of 4 and the block is 16-byte aligned
  const bool y4 = (q & 3) == 0 && (reinterpret_cast<uintptr_t>(reinterpret_cast<float*>(prm.dst) + sq.y_off) & 15) == 0;

  f32x4 acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < ni; i0 += U) {
    // the G_j operands are read from LDS at every group: an offset the
    // compiler cannot see through keeps it from hoisting them all into
    // registers (NL KS 4 VGPRs)
    int gz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(gz));
    const bf16x8* gsv = gs + gz;
    // D u of the group's blocks (their u arrived with the x blocks)
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int m = 0; m < PM; ++m)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(da[m], u_val(uw[u][m], i0 + u, m), acc[u], 0, 0, 0);
      for (int m = PM; m < pm; ++m)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(d_at(m), u_val(u_word(i0 + u, m), i0 + u, m), acc[u], 0, 0, 0);
    }
    // the group's U blocks as B operands (BF16, rounded to nearest even from
    // FP32 state); their ring slots take the next group's blocks at once,
    // after the next group's u
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
    // G_j x_{i0+u} into the partial outputs of block i0 + u + j, each step of
    // G_j read once for the U blocks; lags in fours, a four skipped when
    // every block it would reach lies past the column's end
#pragma unroll
    for (int jq = 0; jq < NL / 4; ++jq) {
      if (i0 + 4 * jq < ni) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int j = 4 * jq + jj;
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const bf16x8 a = gsv[(j * KS + t) * 64 + lane];
#pragma unroll
            for (int u = 0; u < U; ++u)
              acc[u + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[u][t], acc[u + j], 0, 0, 0);
          }
        }
        // the reads run four steps ahead of the MFMAs that use them
        constexpr int NR = 4 * KS;  // reads of the four lags
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int k = 0; k < NR - 4; ++k) {
          __builtin_amdgcn_sched_group_barrier(0x008, U, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * U, 0);
      }
    }
    // the group's blocks are complete: y (outputs 4 g + v of row r)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      const int l = (i << k0) + 16 * c + r;
      const f32x4 y = acc[u];
      if (y4) {
        const uint32_t yoff = i < ni && l < L && 4 * g < q ? (uint32_t)(l * q + 4 * g) * 4u : 0x80000000u;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, y), ry, yoff, 0, 0);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int oo = 4 * g + v;
          const uint32_t yoff = i < ni && l < L && oo < q ? (uint32_t)(l * q + oo) * 4u : 0x80000000u;
          const float yv = y[v];  // (a bit cast of the element itself reads element 0)
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, yv), ry, yoff, 0, 0);
        }
      }
    }
    // shift the partial sums down by U
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = a + U < NA ? acc[a + U] : f32x4{0.f, 0.f, 0.f, 0.f};
  }
}

template <int MP, int S, bool XB>
static hipError_t launch_fold_t(const StageParams& prm, const FoldUnit* units, int n_units, size_t lds,
                                hipStream_t s) {
  {
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_output_fold<MP, S, XB>), (size_t)(160 * 1024));
    if (e != hipSuccess) return e;
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
  (void)p;
  (void)q;
  return (size_t)(1 << s) * (mp / 32) * 64 * 16;  // the G_j
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
