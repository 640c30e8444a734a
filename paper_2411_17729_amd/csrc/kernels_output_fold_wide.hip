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
constexpr int kWideNw = 8;             // waves: eight lags each
constexpr int kWideU = 4;              // blocks per group
constexpr int kWideRing = 64 + kWideU; // output slots in flight
constexpr int kWideMaxP = 64;
// u staging: the rows of one block (16 p elements of 4 bytes, or of 2 bytes
// after a lead of at most 2), in 16-byte chunks
constexpr int kWideUChunks = 16 * kWideMaxP * 4 / 16;
constexpr size_t kWideXs = (size_t)2 * kWideU * kWideKs * 64 * 16;  // two groups of operand blocks
constexpr size_t kWideRingB = (size_t)kWideRing * 32 * 16;
constexpr size_t kWideUs = (size_t)2 * kWideU * kWideUChunks * 16;
constexpr size_t kWideDs = (size_t)8 * kWideMaxP * 4;
constexpr size_t kWideSink = (size_t)64 * 16;  // where threads without a u chunk write theirs
constexpr size_t kWideLds = kWideXs + kWideRingB + kWideUs + kWideDs + kWideSink;
}  // namespace

// Y4: y leaves in 16-byte stores (q a multiple of 4, y 16-byte aligned).
// Every wave issues the same vector memory instructions in the same order on
// every path (loads and stores with nothing to move get an offset past the
// buffer's end, bit 31 set by arithmetic rather than chosen by a branch), so
// the compiler's counter waits are exact.
// Lanes 0..31 of the result hold x of lanes 32..63 (v_permlane32_swap of
// gfx950 exchanges the upper half of its first operand with the lower half of
// its second; s_nop 1 covers the VALU-write-to-permlane-read hazard, which
// the compiler does not see through an asm statement).
__device__ __forceinline__ float upper_half_down(float x) {
  uint32_t a = __float_as_uint(x), b = a;
  asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  return __uint_as_float(b);
}

// Y4: y leaves in 16-byte stores (q a multiple of 4, y 16-byte aligned); UL:
// 16-byte u loads per thread and group (1 while a group's u rows fit 512
// chunks, else 2). Every wave issues the same vector memory instructions in
// the same order on every path (loads and stores with nothing to move get an
// offset past the buffer's end, bit 31 set by arithmetic rather than chosen
// by a branch), and the prologue issues them as a group would, so the
// compiler's counter waits are exact.
template <bool XB, bool Y4, int UL>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_output_fold_wide(
    StageParams prm, const FoldUnit* units) {
  constexpr int MP = kWideMp, KS = kWideKs, U = kWideU, R = kWideRing;
  constexpr int NPW = 4;             // paired operands of a wave (8 lags)
  constexpr int NA = U + 2 * NPW;    // accumulators, offsets -1 .. U + 2 NPW - 2
  constexpr int ES = XB ? 2 : 4;     // bytes of a state entry
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_foldw[];
  bf16x8* xs = reinterpret_cast<bf16x8*>(smem_foldw);                          // [2][U][KS][64]
  f32x4* outs = reinterpret_cast<f32x4*>(smem_foldw + kWideXs);                // [R][32]
  unsigned char* us = smem_foldw + kWideXs + kWideRingB;                       // [2][U][chunks][16]
  float* ds = reinterpret_cast<float*>(smem_foldw + kWideXs + kWideRingB + kWideUs);  // D, q x p
  unsigned char* sink = smem_foldw + kWideXs + kWideRingB + kWideUs + kWideDs;

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
  if (no <= 0) return;  // (the whole workgroup)
  // Lag range of the wave: lags 8 lam .. 8 lam + 7. A lag range is busy in
  // the groups before block no - 8 lam, so lag ranges 0..7 carry decreasing
  // work; waves w and w + 4 share a SIMD, and pairing range w with range
  // 7 - w gives every SIMD the same number of busy groups.
  const int lam = wave < 4 ? wave : 11 - wave;
  // lag ranges 4 .. 7 form D u of a group's output blocks 0 .. 3
  const int du_blk = lam - 4;
  const bool du_wave = du_blk >= 0;

  // this wave's paired operands (lags 8 lam .. + 7) in registers
  bf16x8 ga[NPW][KS];
  {
    const bf16x8* gsrc = reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(prm.P) + o.fold_gc);
#pragma unroll
    for (int i = 0; i < NPW; ++i)
#pragma unroll
      for (int t = 0; t < KS; ++t) ga[i][t] = gsrc[((NPW * lam + i) * KS + t) * 64 + lane];
  }
  for (int e = threadIdx.x; e < R * 32; e += 512) outs[e] = f32x4{0.f, 0.f, 0.f, 0.f};
  {
    const float* dm = reinterpret_cast<const float*>(prm.small) + o.dmat;
    for (int e = threadIdx.x; e < q * p; e += 512) ds[e] = dm[e];
  }

  // state staging: thread s holds operand chunk s of a block (step t = s / 64,
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
  // offset off if on, else off with bit 31 set: past every buffer's end
  // (offsets are below 2^31), so nothing moves
  auto sel = [](bool on, uint32_t off) { return off | ((uint32_t)!on << 31); };
  auto boff = [&](int i) -> uint32_t {
    return sel(i < no, soff + (uint32_t)((i << k0) + 16 * c) * (uint32_t)(MP * ES));
  };

  // u staging: the 16 rows of a block are 16 p contiguous elements; they are
  // copied as 16-byte chunks from the 4-byte-aligned address at or below the
  // first one, so the rows start ulead bytes into the staged copy (block rows
  // start at even rows, so the lead is the same for every block)
  const bool ubf = prm.src_dtype != DT_F32;
  const uint32_t esz = ubf ? 2u : 4u;
  const unsigned char* ub = reinterpret_cast<const unsigned char*>(prm.src) + sq.u_off * esz;
  const uint32_t ulead = (uint32_t)(reinterpret_cast<uintptr_t>(ub) & 3);
  const auto ru = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(ub - ulead), (short)0,
                                                    (int)((ulead + (uint32_t)L * (uint32_t)p * esz + 3u) & ~3u),
                                                    kBufferWord3);
  const int nch = (int)(ulead + 16u * (uint32_t)p * esz + 15u) / 16;  // chunks of one block
  auto uoff = [&](int i, int j) -> uint32_t {  // chunk j of block i
    const uint32_t first = ulead + ((uint32_t)(i << k0) + 16u * (uint32_t)c) * (uint32_t)p * esz;
    return sel(i < no, (first & ~3u) + 16u * (uint32_t)j);
  };
  // chunk j of this thread: block ubk(j) of a group, chunk uci(j) of it
  auto ubk = [&](int j) { return (threadIdx.x + 512 * j) / nch; };
  auto uci = [&](int j) { return (int)(threadIdx.x + 512 * j) - ubk(j) * nch; };
  // its LDS address in u buffer buf (the sink for threads without one, so
  // that every thread writes and no load is moved into a branch)
  auto uslot = [&](int buf, int j) -> unsigned char* {
    return ubk(j) < U ? us + ((size_t)(buf * U + ubk(j)) * kWideUChunks + uci(j)) * 16 : sink + 16 * lane;
  };

  // one group in flight in registers: the state of group gi and the u rows
  // of group gi + 1 (for D u, formed a group ahead)
  f32x4 stf[U][2];  // FP32 state
  u32x4 sth[U];     // BF16 state
  u32x4 uch[UL];
  auto load_group = [&](int gi) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t off = boff(gi * U + u);
      if constexpr (XB) {
        sth[u] = __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0);
      } else {
        stf[u][0] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0));
        stf[u][1] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off + 16, 0, 0));
      }
    }
#pragma unroll
    for (int j = 0; j < UL; ++j)
      uch[j] = __builtin_amdgcn_raw_buffer_load_b128(
          ru, sel(ubk(j) < U, uoff((gi + 1) * U + min(ubk(j), U - 1), uci(j))), 0, 0);
  };
  // the registers into operand buffer buf and u buffer ubuf (the u rows of
  // group j live in u buffer (j + 1) % 2)
  auto write_group = [&](int buf, int ubuf) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bf16x8 v;
      if constexpr (XB) {
        v = __builtin_bit_cast(bf16x8, sth[u]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e] = (__bf16)stf[u][0][e];  // round to nearest even
          v[4 + e] = (__bf16)stf[u][1][e];
        }
      }
      xs[(buf * U + u) * KS * 64 + schunk] = v;
    }
#pragma unroll
    for (int j = 0; j < UL; ++j) *reinterpret_cast<u32x4*>(uslot(ubuf, j)) = uch[j];
  };

  // D u of output block ob (its u rows at ur) added to its ring slot: FP32
  // MFMA 16 x 16 x 4, D's rows as A (zero from q on), u as B (zero for
  // columns from p on). The first PM steps (p <= 4 PM) have D in registers
  // and their LDS reads issued before the first MFMA; wider inputs take
  // further steps from LDS.
  constexpr int PM = 2;
  const int pm = (p + 3) / 4;
  float da[PM];  // (read from LDS once D is staged)
  auto u_at = [&](const unsigned char* ur, int m) {
    const int col = 4 * m + g, cc = min(col, p - 1);  // (columns from p on read column p - 1)
    float uv;
    if (ubf) {
      uv = __uint_as_float((uint32_t)(*reinterpret_cast<const uint16_t*>(ur + (r * p + cc) * 2)) << 16);
    } else {
      uv = *reinterpret_cast<const float*>(ur + (r * p + cc) * 4);
    }
    return col < p ? uv : 0.f;
  };
  auto du_add = [&](int ob, const unsigned char* ur) {
    float uv[PM];
#pragma unroll
    for (int m = 0; m < PM; ++m) uv[m] = u_at(ur, m);
    f32x4 d = g < 2 && ob < no ? outs[(ob % R) * 32 + lane] : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < PM; ++m) d = __builtin_amdgcn_mfma_f32_16x16x4f32(da[m], uv[m], d, 0, 0, 0);
    for (int m = PM; m < pm; ++m) {
      const float dm_ = r < q && 4 * m + g < p ? ds[r * p + 4 * m + g] : 0.f;
      d = __builtin_amdgcn_mfma_f32_16x16x4f32(dm_, u_at(ur, m), d, 0, 0, 0);
    }
    if (g < 2 && ob < no) outs[(ob % R) * 32 + lane] = d;
  };
  // u rows of group j live in u buffer (j + 1) % 2; this wave's D u block of
  // group j
  auto du_group = [&](int j) {
    du_add(j * U + du_blk, us + (size_t)(((j + 1) & 1) * U + du_blk) * kWideUChunks * 16 + ulead);
  };

  float* ydst = reinterpret_cast<float*>(prm.dst) + sq.y_off;
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(ydst, (short)0, (int)((uint32_t)L * (uint32_t)q * 4u), kBufferWord3);
  auto store_y = [&](const f32x4& y, int l, bool ok) {
    const uint32_t lq = (uint32_t)min(l, L - 1) * (uint32_t)q;
    if constexpr (Y4) {
      const uint32_t yoff = sel(ok && l < L && 4 * g < q, (lq + 4u * g) * 4u);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, y), ry, yoff, 0, 0);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int oo = 4 * g + v;
        const uint32_t yoff = sel(ok && l < L && oo < q, (lq + (uint32_t)oo) * 4u);
        const float yv = y[v];  // (a bit cast of the element itself reads element 0)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, yv), ry, yoff, 0, 0);
      }
    }
  };

  // prologue, with the memory operations in the order of a group: the u rows
  // of group 0, then group 0 (with the u rows of group 1) into the
  // registers, out to the buffers, group 1 into the registers, then the y
  // stores of a group (nothing stored here; distinct rows keep them apart)
  u32x4 uch0[UL];
#pragma unroll
  for (int j = 0; j < UL; ++j)
    uch0[j] = __builtin_amdgcn_raw_buffer_load_b128(ru, sel(ubk(j) < U, uoff(min(ubk(j), U - 1), uci(j))), 0, 0);
  load_group(0);
#pragma unroll
  for (int j = 0; j < UL; ++j) *reinterpret_cast<u32x4*>(uslot(1, j)) = uch0[j];
  write_group(0, 0);
  load_group(1);
#pragma unroll
  for (int u = 0; u < U; ++u) store_y(f32x4{0.f, 0.f, 0.f, 0.f}, u, false);
  __syncthreads();  // ring zero, D, group 0 and the u rows of groups 0 and 1 staged
#pragma unroll
  for (int m = 0; m < PM; ++m) da[m] = r < q && 4 * m + g < p ? ds[r * p + 4 * m + g] : 0.f;
  if (du_wave) du_group(0);
  __syncthreads();  // D u of group 0 in its slots

  f32x4 acc[NA];  // acc[a]: output offset a - 1 (top rows), a (bottom rows), from i0 + 8 lam
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ngr = (no + U - 1) / U;
  for (int gi = 0; gi < ngr; ++gi) {
    const int i0 = gi * U, buf = gi & 1;
    if (i0 + 8 * lam < no) {
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
    // group gi + 1 and the u rows of gi + 2 out to the other buffers, then
    // group gi + 2 into the registers (a group of time to arrive)
    write_group(buf ^ 1, buf ^ 1);
    load_group(gi + 2);
    // outputs i0 + 8 lam + u are complete for this wave's lags: top rows of
    // accumulator u + 1 and bottom rows (lanes 32 .. 63, moved to lanes
    // 0 .. 31) of accumulator u; range 0 finishes them into y, the others
    // add into their slots (every other part of these slots was added
    // before the last barrier)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ob = i0 + 8 * lam + u;
      f32x4 val;
#pragma unroll
      for (int v = 0; v < 4; ++v) val[v] = acc[u + 1][v] + upper_half_down(acc[u][v]);
      const bool ok = g < 2 && ob < no;
      const f32x4 sum = (ok ? outs[(ob % R) * 32 + lane] : f32x4{0.f, 0.f, 0.f, 0.f}) + val;
      if (ok) outs[(ob % R) * 32 + lane] = lam != 0 ? sum : f32x4{0.f, 0.f, 0.f, 0.f};
      store_y(sum, (ob << k0) + 16 * c + r, ok && lam == 0);
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = a + U < NA ? acc[a + U] : f32x4{0.f, 0.f, 0.f, 0.f};
    // D u of the next group's outputs
    if (du_wave) du_group(gi + 1);
    __syncthreads();
  }
}

template <bool XB, bool Y4, int UL>
static hipError_t launch_wide_t(const StageParams& prm, const FoldUnit* units, int n_units, hipStream_t s) {
  {
    hipError_t e =
        ensure_dynamic_lds(reinterpret_cast<const void*>(&k_output_fold_wide<XB, Y4, UL>), (size_t)(160 * 1024));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_output_fold_wide<XB, Y4, UL>), dim3(n_units), dim3(512), fold_wide_lds(), s, prm, units);
  return hipGetLastError();
}

template <bool XB, bool Y4>
static hipError_t launch_wide_u(bool ul1, const StageParams& prm, const FoldUnit* units, int n_units, hipStream_t s) {
  return ul1 ? launch_wide_t<XB, Y4, 1>(prm, units, n_units, s) : launch_wide_t<XB, Y4, 2>(prm, units, n_units, s);
}

bool fold_wide_supported(int mp, int ct, int q, int p) {
  return ct == DT_BF16 && mp == kWideMp && q >= 1 && q <= 8 && p >= 1 && p <= kWideMaxP;
}

size_t fold_wide_lds() { return kWideLds; }

hipError_t launch_output_fold_wide(int mp, int ct, bool xb, int max_p, bool q4, const StageParams& prm,
                                   const FoldUnit* units, int n_units, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  if (mp != kWideMp || ct != DT_BF16 || prm.adjoint || max_p < 1 || max_p > kWideMaxP) return hipErrorInvalidValue;
  // 16-byte y stores: every q and y offset a multiple of 4, y 16-byte aligned
  const bool y4 = q4 && (reinterpret_cast<uintptr_t>(prm.dst) & 15) == 0;
  // a group's u rows (FP32, the wider input type, plus a lead) in one chunk per thread
  const bool ul1 = kWideU * ((16 * max_p * 4 + 2 + 15) / 16) <= 512;
  if (xb) return y4 ? launch_wide_u<true, true>(ul1, prm, units, n_units, st)
                    : launch_wide_u<true, false>(ul1, prm, units, n_units, st);
  return y4 ? launch_wide_u<false, true>(ul1, prm, units, n_units, st)
            : launch_wide_u<false, false>(ul1, prm, units, n_units, st);
}

}  // namespace ssmc
