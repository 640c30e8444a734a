// Input pass with the state entries split over the waves (BF16, padded m of
// 128 and 256, p a multiple of 4).
//
// After stages 0..j-1 the state is x_l = K_j w_l with
//   K_j = [Bbar, Abar Bbar, ..., Abar^(2^j - 1) Bbar],  w_l = [u_l; u_{l-1}; ...; u_{l-2^j+1}]
// (zero before the start): the product of the first j factors of eq. (2.2)
// applied to Bbar (§3, first display and eqs. (3.2)-(3.3)). K_j has 2^j p
// columns. The resident input pass keeps K_j in LDS and takes up to m of
// them; here wave w owns state entries w m/8 .. (w+1) m/8 - 1 and keeps the
// rows of K_j for them in registers as MFMA A operands, which takes up to 2 m
// columns (one more folded stage; 128 VGPRs for 512 columns at m = 256). A
// workgroup takes a range of rows of one sequence, stages the range's inputs
// (and the 2^j - 1 before it) once in LDS in BF16, the operand type, with the
// rows in reverse time order so that the window w_l of every row is one
// contiguous run, and then computes its 16-row blocks with no further
// synchronisation: block rows are the MFMA columns, window entries the
// contraction, and a lane's operand is 16 (8 | p) or twice 8 (p = 4)
// contiguous bytes of LDS. The kernel is specialised on the number of MFMA
// steps (2^j p of 128, 256 or 512) and the operand width; each step's operand
// register takes the next block's operand right after its MFMAs, so that the
// LDS reads overlap the MFMAs. The window of a row 16 rows on is the window
// of the row shifted by 16 p entries, i.e. p / 2 MFMA steps (SH): step s >= SH
// of a block takes the operand of step s - SH of the block before, so with
// SH < KS the operands live in a ring of KS + SH registers and a block reads
// only SH of them from LDS (KS / SH times fewer LDS reads), a block ahead of
// their use. The state it writes is FP32, or BF16 (XB, rounded once from the
// FP32 accumulators).
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

template <int MP>
struct InputCfg {
  static constexpr int NW = 8;          // waves of a workgroup
  static constexpr int DW = MP / NW;    // state entries of a wave
  static constexpr int NT = DW / 16;    // MFMA output tiles of a wave
};

// KS: MFMA steps (2^j p / 32); V16: 8 | p (one 16-byte operand read; else p =
// 4); XB: BF16 state; SH: p / 2 when operands are reused across blocks (SH <
// KS, SH divides KS), else 0
template <int MP, int KS, bool V16, bool XB, int SH>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_input_split(
    StageParams prm, const ResRange* units) {
  using C = InputCfg<MP>;
  constexpr int NT = C::NT;
  constexpr int ES = XB ? 2 : 4;  // bytes of a state entry in HBM
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_in[];
  __bf16* us = reinterpret_cast<__bf16*>(smem_in);

  const ResRange rg = units[blockIdx.x];
  const SeqDev sq = prm.seqs[rg.seq];
  const OpDev o = prm.ops[sq.op];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  // 32-bit indices: the host keeps L MP 4 <= 2^31
  const int L = (int)sq.L, p = sq.p;
  const int lag = (1 << sq.kry) - 1;  // rows of input before a row that its window reaches
  const int hi = rg.row0 + rg.nrows;        // rows row0 .. hi - 1 of this unit

  // rows of K_j owned by this wave, A operands: row index r of output tile t
  // is state entry ent(t, r), and a lane's accumulators are the entries
  // ent(t, 4 g) .. + 3 of its time row. FP32 state: ent(t, r) = wave DW +
  // 16 t + r (entries 16 t + 4 g .. + 3, 64 contiguous bytes of a row per
  // store); BF16 state: ent(t, r) = wave DW + 4 NT (r / 4) + 4 t + r mod 4
  // (the lane's tiles are 4 NT contiguous entries, one store). Step s, lane
  // group g holds columns 32 s + 8 g .. + 7.
  auto ent = [&](int t, int rr) {
    return XB ? wave * C::DW + 4 * NT * (rr >> 2) + 4 * t + (rr & 3) : wave * C::DW + 16 * t + rr;
  };

  // inputs of rows row0 - lag .. hi - 1 into LDS, row l at (hi - 1 - l) p,
  // rounded to BF16 (zeros before the start); four channels per element
  // group, eight groups per thread loaded before any is stored. The loads of
  // the first eight groups go out before those of the K_j rows, so that the
  // two latencies overlap and the staging waits for its own loads only.
  const int n4 = (rg.nrows + lag) * p / 4;
  const int64_t ubase = sq.u_off + (int64_t)(rg.row0 - lag) * p;  // element of the first row
  const bool vec = src4_aligned(prm.src, prm.src_dtype, sq.u_off);  // p is a multiple of 4
  f32x4 v[8];
  auto load_groups = [&](int e0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + 512 * i + threadIdx.x, row = rg.row0 - lag + 4 * e / p;
      v[i] = e < n4 && row >= 0 && row < L ? load_src4(prm.src, prm.src_dtype, ubase + 4 * e, vec)
                                          : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto store_groups = [&](int e0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + 512 * i + threadIdx.x;
      if (e < n4) {
        const int flat = 4 * e, row = rg.row0 - lag + flat / p, ch = flat % p;
        bf16x4 b;
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = (__bf16)v[i][c];  // round to nearest even
        *reinterpret_cast<bf16x4*>(us + (hi - 1 - row) * p + ch) = b;
      }
    }
  };
  load_groups(0);
  __builtin_amdgcn_sched_barrier(0);
  bf16x8 ka[NT][KS];
  {
    const __bf16* K = reinterpret_cast<const __bf16*>(prm.P) + o.kc;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s)
        ka[t][s] = *reinterpret_cast<const bf16x8*>(K + (int64_t)ent(t, r) * o.kst + 32 * s + 8 * g);
  }
  __builtin_amdgcn_sched_barrier(0);
  store_groups(0);
  for (int e0 = 8 * 512; e0 < n4; e0 += 8 * 512) {
    load_groups(e0);
    store_groups(e0);
  }
  __syncthreads();

  // x^(j) rows through a buffer resource over the sequence's L x MP block
  // (stores of rows past L are dropped); buffer kry mod 2 as for the resident
  // input pass
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  unsigned char* xo =
      reinterpret_cast<unsigned char*>((sq.kry & 1) ? prm.xout : const_cast<void*>(prm.xin)) + sq.x_off * ES;
  const auto rout = __builtin_amdgcn_make_buffer_rsrc(xo, (short)0, (int)nrec, kBufferWord3);
  const uint32_t lane_off = (uint32_t)(r * MP + ent(0, 4 * g)) * (uint32_t)ES;
  const int nblk = (rg.nrows + 15) / 16;
  // operand of step s for block b: this lane's row l = row0 + 16 b + r has its
  // window at (hi - 1 - l) p; rows past the unit read staged rows of the unit's
  // end (their outputs are not stored)
  auto operand = [&](int b, int s) -> bf16x8 {
    const int l = rg.row0 + 16 * b + r;
    const int w0 = (l < hi ? hi - 1 - l : 0) * p + 8 * g + 32 * s;
    if constexpr (V16) {
      return *reinterpret_cast<const bf16x8*>(us + w0);
    } else {
      const bf16x4 lo = *reinterpret_cast<const bf16x4*>(us + w0);
      const bf16x4 up = *reinterpret_cast<const bf16x4*>(us + w0 + 4);
      return __builtin_shufflevector(lo, up, 0, 1, 2, 3, 4, 5, 6, 7);
    }
  };
  auto store_block = [&](int b, const f32x4(&acc)[NT]) {
    const int l = rg.row0 + 16 * b + r;
    const uint32_t off = l < hi ? lane_off + (uint32_t)(16 * b + rg.row0) * (uint32_t)(MP * ES) : 0x80000000u;
    if constexpr (!XB) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, acc[t]), rout, off + 64 * t, 0, 0);
    } else {
      bf16x8 xb;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) xb[4 * t + e] = (__bf16)acc[t][e];  // round to nearest even
      const u32x4 w4 = __builtin_bit_cast(u32x4, xb);
      if constexpr (NT == 2) {
        __builtin_amdgcn_raw_buffer_store_b128(w4, rout, off, 0, 0);
      } else {
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{w4[0], w4[1]}, rout, off, 0, 0);
      }
    }
  };
  bf16x8 bo[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) bo[s] = operand(0, s);
  if constexpr (SH == 0) {
    for (int b = 0; b < nblk; ++b) {
      // each step's operand register takes the next block's operand right
      // after its MFMAs, so the LDS reads of a block overlap the MFMAs of the
      // one before
      f32x4 acc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[t][s], bo[s], acc[t], 0, 0, 0);
        bo[s] = operand(b + 1, s);
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);           // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, V16 ? 1 : 2, 0);  // DS read
      }
      store_block(b, acc);
    }
  } else {
    // operand ring of KS + SH registers: step s of block b sits in register
    // (s - b SH) mod (KS + SH). The SH registers block b does not use take
    // the next block's first SH operands (read from LDS at the start of block
    // b, a block ahead of use); the rest of the next block's operands are
    // this block's. NR blocks bring the ring back to its start. A block's
    // accumulators are rounded and stored after the next block's MFMAs are
    // issued (two accumulator sets), so no wave waits for its own results.
    constexpr int RG = KS + SH, NR = RG / SH, NR2 = 2 * NR;
    static_assert(SH > 0 && KS % SH == 0 && KS > SH, "operand reuse needs SH < KS dividing KS");
    bf16x8 ring[RG];
#pragma unroll
    for (int s = 0; s < KS; ++s) ring[s] = bo[s];
    f32x4 acc[2][NT];
    for (int b0 = 0; b0 < nblk; b0 += NR2) {
#pragma unroll
      for (int rr = 0; rr < NR2; ++rr) {
        const int b = b0 + rr;
        if (b < nblk) {
          // the next block's first SH operands into the registers this block
          // leaves free
#pragma unroll
          for (int i = 0; i < SH; ++i) ring[(i - (rr + 1) * SH + NR2 * RG) % RG] = operand(b + 1, i);
          __builtin_amdgcn_sched_barrier(0);  // (left alone, the reads sink to the block's end)
          f32x4(&a)[NT] = acc[rr & 1];
#pragma unroll
          for (int t = 0; t < NT; ++t) a[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const bf16x8 bop = ring[(s - rr * SH + NR2 * RG) % RG];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[t][s], bop, a[t], 0, 0, 0);
          }
          if (b > 0) store_block(b - 1, acc[(rr + 1) & 1]);
        }
      }
    }
    if (nblk > 0) {
      if ((nblk - 1) & 1)
        store_block(nblk - 1, acc[1]);
      else
        store_block(nblk - 1, acc[0]);
    }
  }
}

template <int MP, int KS, bool V16, bool XB, int SH>
static hipError_t launch_input_t(const StageParams& prm, const ResRange* units, int n_units,
                                 size_t lds, hipStream_t s) {
  {
    hipError_t e =
        ensure_dynamic_lds(reinterpret_cast<const void*>(&k_input_split<MP, KS, V16, XB, SH>), (size_t)(65536));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_input_split<MP, KS, V16, XB, SH>), dim3(n_units), dim3(512), lds, s, prm, units);
  return hipGetLastError();
}

// operand reuse across blocks (SH = p / 2 steps) where the window spans more
// than one block of rows: p = 4 (two 8-byte reads per operand) shifts by 2
// steps, p = 8 by 4, p = 16 by 8
template <int MP, int KS, bool XB>
static hipError_t launch_input_x(int p, const StageParams& prm, const ResRange* units, int n_units, size_t lds,
                                 hipStream_t s) {
  if (p == 4) {
    if constexpr (KS > 2) return launch_input_t<MP, KS, false, XB, 2>(prm, units, n_units, lds, s);
    return launch_input_t<MP, KS, false, XB, 0>(prm, units, n_units, lds, s);
  }
  if (p == 8) {
    if constexpr (KS > 4) return launch_input_t<MP, KS, true, XB, 4>(prm, units, n_units, lds, s);
    return launch_input_t<MP, KS, true, XB, 0>(prm, units, n_units, lds, s);
  }
  if (p == 16) {
    if constexpr (KS > 8) return launch_input_t<MP, KS, true, XB, 8>(prm, units, n_units, lds, s);
    return launch_input_t<MP, KS, true, XB, 0>(prm, units, n_units, lds, s);
  }
  return launch_input_t<MP, KS, true, XB, 0>(prm, units, n_units, lds, s);
}

template <int MP, int KS>
static hipError_t launch_input_w(int p, bool xb, const StageParams& prm, const ResRange* units,
                                 int n_units, size_t lds, hipStream_t s) {
  return xb ? launch_input_x<MP, KS, true>(p, prm, units, n_units, lds, s)
            : launch_input_x<MP, KS, false>(p, prm, units, n_units, lds, s);
}

bool input_split_supported(int mp, int ct, int p, int kdim) {
  return ct == DT_BF16 && (mp == 128 || mp == 256) && (p == 4 || (p > 0 && (p & 7) == 0)) &&
         (kdim == 128 || kdim == 256 || (kdim == 512 && mp == 256));
}

hipError_t launch_input_split(int mp, int ct, int p, int kdim, bool xb, const StageParams& prm,
                              const ResRange* units, int n_units, size_t lds, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  if (!input_split_supported(mp, ct, p, kdim) || lds > 65536) return hipErrorInvalidValue;
  if (mp == 128)
    return kdim == 128 ? launch_input_w<128, 4>(p, xb, prm, units, n_units, lds, s)
                       : launch_input_w<128, 8>(p, xb, prm, units, n_units, lds, s);
  return kdim == 128   ? launch_input_w<256, 4>(p, xb, prm, units, n_units, lds, s)
         : kdim == 256 ? launch_input_w<256, 8>(p, xb, prm, units, n_units, lds, s)
                       : launch_input_w<256, 16>(p, xb, prm, units, n_units, lds, s);
}

}  // namespace ssmc
