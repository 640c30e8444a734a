// Two consecutive lean stages of the forward cascade in one pass over the state.
//
// Stages k and k+1 are two factors of the product of §2 (eq. (2.2)) applied as
// in §3: with y_l = x_l + P_k x_{l-2^k} they give
//   w_l = y_l + P_{k+1} y_{l-2^{k+1}},  P_{k+1} = P_k^2.
// In the column numbering of stage k (16-row blocks spaced 2^k apart; block i
// of column c holds rows i 2^k + 16 c + r, r < 16) the stage-k partner of
// block i is block i - 1 of the same column and the stage-(k+1) partner is
// block i - 2. A workgroup walks T consecutive blocks of the numbering. Its
// eight waves split the state entries, wave w owning entries w m/8 .. (w+1)
// m/8 - 1, and keep the rows of P_k and P_{k+1} for them in registers as MFMA
// A operands; the time rows of a block are the MFMA columns. A block's y needs
// every wave's share of the previous block's x, and its w the y of two blocks
// back, so both are exchanged through LDS in BF16, the operand type of the
// per-stage kernels (which round the FP32 stage input the same way). Three
// warm-up blocks before the segment, inside its column, rebuild those
// partners: a segment reads T + 3 blocks (fewer at a column start) and writes
// T, for two stages.
//
// Each block's rows are loaded DP blocks ahead into registers; one barrier
// per block orders the LDS exchange. The exchange runs one block ahead: a
// block is contracted with partners read during the previous visit, and each
// operand register, once its MFMAs are issued, is refilled with the same
// piece of the next block's partner (x of this block, y of the previous one,
// both complete since the last barrier), so the LDS reads overlap the MFMAs;
// x of the next block goes to its slot during the visit. x and y of block i
// take slot i mod 2 of two buffers each.
//
// The tail variant runs the last two stages of every sequence of the launch
// and forms y_l = C w_l + D u_l (last display of §3; eq. (1.2)) instead of
// storing w. Since C w_l = C y_l + (C P_{k+1}) y_{l-2^{k+1}}, the second stage
// needs no m x m contraction: with the q x m product C P_{k+1} formed once
// (FP64, then rounded to the operand type), each wave contracts its share of
// y (FP32 MFMA, C's columns in registers) and its share of the y two blocks
// back (one MFMA against its columns of C P_{k+1}); the eight partial outputs
// of a block meet in LDS (two buffers, so that a block's partials are added up
// during the next block, behind the same barrier), and wave v adds them for
// rows 2v and 2v+1 with D u_l. The D u_l of the segment's rows are formed at
// the start into LDS, so that no load in the walk is waited for out of order.
//
// The state between passes is FP32, or BF16 (XB): then the rows are loaded and
// stored as BF16, x goes to LDS as loaded, and y and w are still accumulated
// in FP32 and rounded once, when they are written.
#include "stage_common.h"
#include "ssm_internal.h"

namespace ssmc {

template <int MP>
struct PairCfg {
  static constexpr int NW = 8;             // waves of a workgroup
  static constexpr int DW = MP / NW;       // state entries of a wave
  static constexpr int NT = DW / 16;       // MFMA output tiles of a wave
  static constexpr int KS = MP / 32;       // MFMA steps of one contraction
  static constexpr int RS = MP + 16;       // LDS row stride in BF16 entries (32-byte pad)
  static constexpr int SLOT = 16 * RS;     // one block of 16 time rows
  static constexpr int DP = 4;             // blocks loaded ahead
  static constexpr size_t LDS = 4 * SLOT * sizeof(__bf16);  // x and y: 2 slots each
  // tail variant: two buffers of partial outputs (8 waves x 16 rows x 16
  // outputs), then D u of the segment's rows, D and the segment's inputs
  // after the slots
  static constexpr size_t RED = 2 * NW * 16 * 16 * sizeof(float);
};

template <int MP, bool TAIL, bool XB>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_stage_pair(
    StageParams prm, const PairUnit* units) {
  using C = PairCfg<MP>;
  constexpr int NT = C::NT, KS = C::KS, DP = C::DP, RS = C::RS, SLOT = C::SLOT;
  constexpr int ES = XB ? 2 : 4;  // bytes of a state entry in HBM
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pair[];
  __bf16* xs = reinterpret_cast<__bf16*>(smem_pair);
  __bf16* ys = xs + 2 * SLOT;

  const PairUnit un = units[blockIdx.x];
  const SeqDev sq = prm.seqs[un.seq];
  const OpDev o = prm.ops[sq.op];
  const int k = prm.k;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;
  // 32-bit indices: the host keeps L MP 4 <= 2^31 and 2^(k+1) < L
  const int L = (int)sq.L;
  const int ni = (L + (1 << k) - 1) >> k;  // blocks per column
  const int nflat = (1 << (k - 4)) * ni;
  const int f0 = un.f0;
  const int f1 = min(f0 + un.T, nflat);
  if (f0 >= f1) return;  // the whole workgroup
  const int c0 = f0 / ni, i0 = f0 - c0 * ni;
  const int nw = min(3, i0);      // warm-up blocks (they stay in the segment's first column)
  const int nit = f1 - f0 + nw;   // blocks visited

  // Rows of P_k and P_{k+1} owned by this wave, as A operands: row index r of
  // output tile t is state entry ent(t, r), so a lane's accumulators are the
  // entries ent(t, 4 g) .. + 3 of its time row. FP32 state: ent(t, r) =
  // wave DW + 16 t + r, entries 16 t + 4 g .. + 3 of the wave's share, and
  // every memory instruction moves 64 contiguous bytes of each row. BF16
  // state: ent(t, r) = wave DW + 4 NT (r / 4) + 4 t + r mod 4, so that the
  // lane's NT tiles are the 4 NT contiguous entries from 4 NT g on and one
  // instruction moves the wave's whole share of each row. Contraction step s
  // covers entries 32 s .. 32 s + 31 with operand slot 8 g + 4 h + e holding
  // entry 32 s + 16 h + 4 g + e, the assignment of the chain kernel, so that
  // every output sees the same products in the same MFMA steps as there.
  // The share of wave w is share wp = w for the first half of the waves and
  // NW - 1 - (w - NW / 2) for the second, so that the two waves of a SIMD (w
  // and w + NW / 2) hold one low and one high share: with a lower-triangular
  // P (every power of a lower-triangular Abar) a share needs the contraction
  // steps up to its last entry only, and the two waves of a SIMD then run
  // about the same number of steps.
  const int wp = wave < C::NW / 2 ? wave : C::NW - 1 - (wave - C::NW / 2);
  // (BF16 state only: with FP32 state the extra branches cost registers the
  // variant does not have)
  const int nsteps = XB && o.lower ? (wp * C::DW + C::DW - 1) / 32 + 1 : KS;  // steps s < nsteps
  auto ent = [&](int t, int rr) {
    return XB ? wp * C::DW + 4 * NT * (rr >> 2) + 4 * t + (rr & 3) : wp * C::DW + 16 * t + rr;
  };
  bf16x8 pa[2][NT][KS];
  // tail: contraction step cps (columns 32 cps .. + 31) of C P_{k+1}, row r:
  // step `wave` for the first KS waves, nothing for the others (padded m 128)
  const int cps = wave < KS ? wave : 0;
  const bool has_cps = wave < KS;
  bf16x8 cpa;
  {
    const __bf16* P0 = reinterpret_cast<const __bf16*>(prm.P) + o.pc + (int64_t)k * MP * MP;
#pragma unroll
    for (int h = 0; h < (TAIL ? 1 : 2); ++h)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const __bf16* row = P0 + (int64_t)h * MP * MP + ent(t, r) * MP + 32 * s + 4 * g;
          const bf16x4 lo = *reinterpret_cast<const bf16x4*>(row);
          const bf16x4 hi = *reinterpret_cast<const bf16x4*>(row + 16);
          pa[h][t][s] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        }
    if constexpr (TAIL) {
      const __bf16* row = reinterpret_cast<const __bf16*>(prm.P) + o.cpc + r * MP + 32 * cps + 4 * g;
      const bf16x4 lo = *reinterpret_cast<const bf16x4*>(row);
      const bf16x4 hi = *reinterpret_cast<const bf16x4*>(row + 16);
      cpa = has_cps ? __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7) : bf16x8{};
    }
  }

  // State rows through buffer resources over the sequence's L x MP block:
  // rows past L read as zero and their stores are dropped; offset 2^31 marks
  // an absent block.
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(reinterpret_cast<const unsigned char*>(prm.xin)) + sq.x_off * ES,
      (short)0, (int)nrec, kBufferWord3);
  const auto rout = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<unsigned char*>(prm.xout) + sq.x_off * ES,
                                                      (short)0, (int)nrec, kBufferWord3);

  // tail: C's columns for this wave's entries as FP32 MFMA A operands (row
  // index r is output r, zero from q on), and D u for the segment's rows
  // (block v of the segment, row rr, output j at (16 v + rr) q + j), formed
  // from the segment's inputs and D staged in LDS (the loads all go out
  // before any is waited for)
  const int q = sq.q, p = sq.p;
  float ca[NT][4];
  float* red = reinterpret_cast<float*>(smem_pair + C::LDS);
  float* du = red + C::RED / sizeof(float);
  if constexpr (TAIL) {
    const float* cm = reinterpret_cast<const float*>(prm.small) + o.cout;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        ca[t][v] = r < q ? cm[r * MP + ent(t, 4 * g + v)] : 0.f;
    const int nv = f1 - f0;
    float* Ds = du + nv * 16 * q;
    float* Us = Ds + ((q * p + 3) & ~3);  // 16-byte aligned
    const float* dm = reinterpret_cast<const float*>(prm.small) + o.dmat;
    for (int e = threadIdx.x; e < q * p; e += 512) Ds[e] = dm[e];
    // the segment's inputs: a block's 16 rows are 16 p contiguous elements;
    // groups of four, eight per thread loaded before any is stored
    const int n4 = nv * 4 * p;
    const bool vec = src4_aligned(prm.src, prm.src_dtype, sq.u_off);  // block starts are 16-row aligned
    for (int e0 = 0; e0 < n4; e0 += 8 * 512) {
      f32x4 v4[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 512 * i + threadIdx.x;
        const int v = e / (4 * p), w = 4 * (e - v * 4 * p);  // block and element within it
        const int f = f0 + v, col = f / ni, row0 = ((f - col * ni) << k) + 16 * col;
        const int64_t gi = sq.u_off + (int64_t)row0 * p + w;
        const bool whole = row0 + (w + 3) / p < L;
        f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
        if (e < n4) {
          if (whole && vec) {
            a = load_src4(prm.src, prm.src_dtype, gi, true);
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
              if (row0 + (w + c) / p < L) a[c] = load_src<float>(prm.src, prm.src_dtype, gi + c);
          }
        }
        v4[i] = a;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 512 * i + threadIdx.x;
        if (e >= n4) break;
        *reinterpret_cast<f32x4*>(Us + 4 * e) = v4[i];
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nv * 16 * q; e += 512) {
      const int vr = e / q, j = e - vr * q;
      float a = 0.f;
      for (int c = 0; c < p; ++c) a += Ds[j * p + c] * Us[vr * p + c];
      du[e] = a;
    }
    __syncthreads();
  }
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float*>(prm.dst) + sq.y_off, (short)0,
                                                    TAIL ? (int)((uint32_t)L * (uint32_t)q * 4u) : 0,
                                                    kBufferWord3);
  // this lane's entries of a block: time row r, from entry ent(0, 4 g) on
  const uint32_t lane_off = (uint32_t)(r * MP + ent(0, 4 * g)) * (uint32_t)ES;
  auto row_off = [&](int col, int i) -> uint32_t {
    return lane_off + (uint32_t)((i << k) + 16 * col) * (uint32_t)(MP * ES);
  };

  // Blocks are loaded DP visits ahead into a ring of registers (FP32 state:
  // a block is accumulated in place); a slot takes the load of the block DP
  // visits later once its block is stored. The visits are padded to a
  // multiple of DP, and loads and stores are issued on every visit (out of
  // range where there is nothing to move), so every path has the same memory
  // operations in flight and the compiler's counter waits stay exact.
  const int npad = (nit + DP - 1) / DP * DP;
  f32x4 xr[DP][NT];   // FP32 state
  u32x4 xh[DP];       // BF16 state, NT = 2: entries 8 g .. + 7
  u32x2 xq[DP];       // BF16 state, NT = 1: entries 4 g .. + 3
  int lc = c0, li = i0 - nw, nl = 0;  // next block to load and how many were issued
  auto issue = [&](int u) {
    const uint32_t off = nl < nit ? row_off(lc, li) : 0x80000000u;
    if constexpr (!XB) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
        xr[u][t] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off + 64 * t, 0, 0));
    } else if constexpr (NT == 2) {
      xh[u] = __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0);
    } else {
      xq[u] = __builtin_amdgcn_raw_buffer_load_b64(rin, off, 0, 0);
    }
    ++nl;
    if (++li == ni) {
      li = 0;
      ++lc;
    }
  };
  // w of a block (lean variant), BF16 rounded to nearest even for XB
  auto store_w = [&](uint32_t off, const f32x4(&acc)[NT]) {
    if constexpr (!XB) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, acc[t]), rout, off + 64 * t, 0, 0);
    } else {
      bf16x8 wb;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) wb[4 * t + e] = (__bf16)acc[t][e];
      const u32x4 w4 = __builtin_bit_cast(u32x4, wb);
      if constexpr (NT == 2) {
        __builtin_amdgcn_raw_buffer_store_b128(w4, rout, off, 0, 0);
      } else {
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{w4[0], w4[1]}, rout, off, 0, 0);
      }
    }
  };
  // The ring is filled as DP visits would fill it, with the stores of a visit
  // (out of range here, so nothing is written) in their place: a lean visit
  // stores w and then loads, a tail visit loads first (its slot is free once
  // the accumulators are set) and stores y at its end. The memory counter then
  // stands at the loop's entry as it does on every later pass, and the
  // compiler's wait for a slot covers that slot's load only.
#pragma unroll
  for (int u = 0; u < DP; ++u) {
    if constexpr (TAIL) {
      issue(u);
      __builtin_amdgcn_raw_buffer_store_b32(0u, ry, 0x80000000u, 0, 0);
    } else {
      f32x4 z[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) z[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      store_w(0x80000000u, z);
      issue(u);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the ring's loads in visit order
  }

  // LDS rows hold a block's entries in operand order: entry n at position
  // 32 (n / 32) + 8 ((n / 4) mod 4) + 4 ((n / 16) mod 2) + n mod 4, so that the
  // B operand of step s is the 16 bytes at 32 s + 8 g of row r. This lane
  // writes its entries of row r as NT groups of four, ent(t, 4 g) .. + 3.
  auto pos = [](int n) { return 32 * (n >> 5) + 8 * ((n >> 2) & 3) + 4 * ((n >> 4) & 1) + (n & 3); };
  int wr[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wr[t] = r * RS + pos(ent(t, 4 * g));
  const int rd = r * RS + 8 * g;
  auto put = [&](__bf16* slot, const f32x4(&v)[NT]) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x4 b;
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = (__bf16)v[t][e];  // round to nearest even
      *reinterpret_cast<bf16x4*>(slot + wr[t]) = b;
    }
  };
  // BF16 state: x of ring slot u goes to LDS as loaded and is widened to FP32
  // as the accumulator of y
  auto put_raw = [&](__bf16* slot, int u) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      u32x2 w2;
      if constexpr (NT == 2) {
        w2 = u32x2{xh[u][2 * t], xh[u][2 * t + 1]};
      } else {
        w2 = xq[u];
      }
      *reinterpret_cast<u32x2*>(slot + wr[t]) = w2;
    }
  };
  auto widen = [&](int u, f32x4(&acc)[NT]) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t w2 = NT == 2 ? xh[u][2 * t + e / 2] : xq[u][e / 2];
        acc[t][e] = __builtin_bit_cast(float, (e & 1) ? (w2 & 0xffff0000u) : (w2 << 16));
      }
  };
  // operands of a visit without that partner are zeros (a select, so stale
  // LDS contents cannot leak in)
  auto keep = [&](bool on, bf16x8(&b)[KS]) {
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = on ? b[s] : bf16x8{};
  };
  // one contraction; operand step s is refilled from the next partner's row
  // (at src) right after its MFMAs
  auto contract_refill = [&](const bf16x8(&a)[NT][KS], bf16x8(&b)[KS], f32x4(&acc)[NT], const __bf16* src) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (s >= nsteps) break;  // the share's entries see no input past its own
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][s], b[s], acc[t], 0, 0, 0);
      b[s] = *reinterpret_cast<const bf16x8*>(src + 32 * s);
    }
  };

  int cc = c0, ci = i0 - nw;  // block being computed
  // x of the first block to its slot; the partners of the first visit are
  // absent (zeros)
  if constexpr (XB) {
    put_raw(xs, 0);
  } else {
    put(xs, xr[0]);
  }
  __syncthreads();
  __builtin_amdgcn_sched_barrier(0);
  bf16x8 b[KS], b2[TAIL ? 1 : KS];  // partners of the visit: x of the previous block, y two back
#pragma unroll
  for (int s = 0; s < KS; ++s) b[s] = bf16x8{};
#pragma unroll
  for (int s = 0; s < (TAIL ? 1 : KS); ++s) b2[s] = bf16x8{};
  // tail: y of a block from its partials (buffer pb) and D u (segment block
  // v), first row l0; wave w takes rows 2w and 2w + 1 (lanes below 32, output
  // lane % 16). gather reads them into registers at the start of a visit,
  // finish stores their sum at its end.
  const int frr = 2 * wave + ((lane >> 4) & 1), fqq = lane & 15;
  auto gather = [&](const float* pb, int v, float(&fin)[C::NW + 1]) {
#pragma unroll
    for (int w = 0; w < C::NW; ++w) fin[w] = pb[(w * 16 + frr) * 16 + fqq];
    fin[C::NW] = du[(v * 16 + frr) * q + (fqq < q ? fqq : 0)];
  };
  auto finish = [&](const float(&fin)[C::NW + 1], int l0, bool has) {
    float yv = 0.f;
#pragma unroll
    for (int w = 0; w <= C::NW; ++w) yv += fin[w];
    const int l = l0 + frr;
    const uint32_t yoff = has && lane < 32 && fqq < q && l < L ? (uint32_t)(l * q + fqq) * 4u : 0x80000000u;
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, yv), ry, yoff, 0, 0);
  };
  int pl0 = 0, pv = 0;  // tail: the previous block's first row and segment index
  bool pout = false;    //       and whether it has outputs
  for (int it0 = 0; it0 < npad; it0 += DP) {
#pragma unroll
    for (int u = 0; u < DP; ++u) {
      const int it = it0 + u;
      const bool real = it < nit;  // padding visits move nothing
      const bool out = real && it >= nw;
      const uint32_t off = out ? row_off(cc, ci) : 0x80000000u;
      // the next visit's partners: x of this block and y of the previous one
      // (tail: only the columns of step cps of that y)
      const __bf16* nx = xs + (it & 1) * SLOT + rd;
      const __bf16* ny = ys + ((it + 1) & 1) * SLOT + rd;
      // tail: the previous block's partials, complete since the last barrier
      float fin[C::NW + 1];
      if constexpr (TAIL) gather(red + ((it + 1) & 1) * (C::NW * 256), pv, fin);
      // x of the next block to its slot
      // the block's accumulators: the ring slot itself (lean, FP32 state) or
      // a copy, after which a tail visit reloads the slot at once
      f32x4 xw[NT];
      f32x4(&acc)[NT] = XB || TAIL ? xw : xr[u];
      if constexpr (XB) {
        put_raw(xs + ((it + 1) & 1) * SLOT, (u + 1) % DP);
        widen(u, xw);
      } else {
        put(xs + ((it + 1) & 1) * SLOT, xr[(u + 1) % DP]);
        if constexpr (TAIL) {
#pragma unroll
          for (int t = 0; t < NT; ++t) xw[t] = xr[u][t];
        }
      }
      if constexpr (TAIL) issue(u);
      // y = x + P_k x_prev (no partner at a column's first block; the first of
      // three warm-up blocks only provides x)
      keep(real && ci >= 1 && it > nw - 3, b);
      contract_refill(pa[0], b, acc, nx);
      put(ys + (it & 1) * SLOT, acc);
      if constexpr (!TAIL) {
        // w = y + P_{k+1} y_prev2
        keep(out && ci >= 2, b2);
        contract_refill(pa[1], b2, acc, ny);
        store_w(off, acc);
        // each step's refill right behind its MFMAs (left to itself the
        // scheduler sinks the reads below the contractions)
#pragma unroll
        for (int i = 0; i < 2 * KS; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);  // MFMA
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
        }
      }
      if constexpr (TAIL) {
        // this wave's part of C w = C y + (C P_{k+1}) y_prev2 (outputs 4 g + v
        // of time row r; one accumulator chain per tile of y) into buffer it
        // mod 2; the previous block's partials become its y
        f32x4 yp[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          yp[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int v = 0; v < 4; ++v) yp[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[t][v], acc[t][v], yp[t], 0, 0, 0);
        }
        f32x4 ya = yp[0];
#pragma unroll
        for (int t = 1; t < NT; ++t) ya += yp[t];
        const bf16x8 yb = has_cps && out && ci >= 2 ? b2[0] : bf16x8{};
        ya = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cpa, yb, ya, 0, 0, 0);
        b2[0] = *reinterpret_cast<const bf16x8*>(ny + 32 * cps);
        *reinterpret_cast<f32x4*>(red + (it & 1) * (C::NW * 256) + (wave * 16 + r) * 16 + 4 * g) = ya;
        finish(fin, pl0, pout);
        pl0 = (ci << k) + 16 * cc;
        pout = out;
        pv = out ? it - nw : 0;
      }
      if constexpr (!TAIL) issue(u);
      __syncthreads();
      // a visit's work stays in it: hoisted, the widening of the next slot
      // would wait for that slot's load a visit early
      __builtin_amdgcn_sched_barrier(0);
      if (++ci == ni) {
        ci = 0;
        ++cc;
      }
    }
  }
  if constexpr (TAIL) {  // the last block
    float fin[C::NW + 1];
    gather(red + ((npad + 1) & 1) * (C::NW * 256), pv, fin);
    finish(fin, pl0, pout);
  }
}

template <int MP, bool TAIL, bool XB>
static hipError_t launch_pair_v(const StageParams& prm, const PairUnit* units, int n_units,
                                size_t lds, hipStream_t s) {
  {
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage_pair<MP, TAIL, XB>), (size_t)(160 * 1024));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_stage_pair<MP, TAIL, XB>), dim3(n_units), dim3(512), lds, s, prm, units);
  return hipGetLastError();
}

template <int MP, bool TAIL>
static hipError_t launch_pair_t(bool xb, const StageParams& prm, const PairUnit* units, int n_units,
                                size_t lds, hipStream_t s) {
  return xb ? launch_pair_v<MP, TAIL, true>(prm, units, n_units, lds, s)
            : launch_pair_v<MP, TAIL, false>(prm, units, n_units, lds, s);
}

bool pair_supported(int mp, int ct) { return ct == DT_BF16 && (mp == 128 || mp == 256); }

size_t pair_lds(int mp, bool tail, int seg_blocks, int p, int q) {
  const size_t base = mp == 128 ? PairCfg<128>::LDS : PairCfg<256>::LDS;
  if (!tail) return base;
  return base + PairCfg<256>::RED + ((size_t)seg_blocks * 16 * (q + p) + (size_t)q * p + 3) * sizeof(float);
}

hipError_t launch_stage_pair(int mp, int ct, const StageParams& prm, const PairUnit* units,
                             int n_units, bool tail, bool xb, size_t lds, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  if (ct != DT_BF16 || prm.adjoint || lds > 160 * 1024) return hipErrorInvalidValue;
  switch (mp) {
    case 128: return tail ? launch_pair_t<128, true>(xb, prm, units, n_units, lds, s)
                          : launch_pair_t<128, false>(xb, prm, units, n_units, lds, s);
    case 256: return tail ? launch_pair_t<256, true>(xb, prm, units, n_units, lds, s)
                          : launch_pair_t<256, false>(xb, prm, units, n_units, lds, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ssmc
