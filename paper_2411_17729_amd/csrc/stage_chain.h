// Chain walk of one stage (device code shared by the per-stage kernel and the
// persistent launch): 16-row blocks spaced by the shift.
//
// Stage k couples the rows l and l - 2^k (§3: x_l <- x_l + P_k x_{l-2^k}; the
// adjoint g_l <- g_l + P_k^T g_{l+2^k}). For 2^k >= 16 the time rows of a
// sequence fall into columns of 16-row blocks: block i of column c holds rows
// i 2^k + 16 c + j, j < 16, and the shifted operand of block i is the stage
// input of block i - 1 of the same column (block i + 1 for the adjoint). Blocks
// are numbered column by column and a wave takes a segment of T consecutive
// numbers; it keeps each block's input rows in registers as the shifted
// operand of the next block, so every state row is read once per stage (plus
// one extra block per segment) rather than twice as in k_stage_res.
//
// The power is resident in LDS as in k_stage_res. The shifted operand now
// arrives in the accumulator layout (a lane holds entries 16 nb + 4 g + v of
// its time row), so the contraction index of each MFMA step is assigned to
// match: for BF16, operand slot 8 g + 4 h + e of step c is state entry
// 16 (2c + h) + 4 g + e, and the LDS copy of the power has its columns
// permuted the same way; for FP32, step (a, t) contracts entry 16 a + 4 g + t,
// which is already the layout.
#pragma once
#include <type_traits>

#include "stage_res.h"

namespace ssmc {

// TAIL: some sequence of the launch ends at this stage (output epilogue or a
// copy of the final state may be due); otherwise the lean variant runs, which
// only stores the stage output. S: segments walked side by side by each wave
// (more loads in flight per wave for small state sizes); the unit covers
// segments seg0 .. seg0 + 8 S - 1, wave w taking seg0 + w S .. seg0 + w S + S - 1.
// When the power does not fit in LDS (FP32, m = 256) two workgroups share a
// unit, each holding half of P_k's rows and producing half of every output
// row: half h the 16-entry pieces 4 i + 2 h and 4 i + 2 h + 1, i < 4, so that
// each stores whole 128-byte lines. Both load whole input rows, which the
// next block needs as its shifted operand. The split form has no output
// epilogue. To keep register indices static, a split workgroup holds its own
// pieces first: register piece e < 8 is row piece 4 (e / 2) + 2 h + e mod 2,
// and register piece 8 + e the other half's 4 (e / 2) + 2 (1 - h) + e mod 2;
// its LDS copy of P_k has the columns permuted the same way, so MFMA step a
// still pairs register piece a with the matching columns.
//
// TRI (FP32): 1 when every power of the launch is lower triangular (the
// adjoint's P_k^T upper triangular: TRI 2), and the contraction leaves out the
// 16 x 16 blocks that are zero; the host chooses it, so the unrolled loop has
// no branches. Output piece o needs input pieces up to o (from o for the
// adjoint). For its e-th own piece a half takes its own register pieces
// a <= e (>= e for the adjoint) and the other half's pieces 8 + a with
// a / 2 <= e / 2 (>= for the adjoint): one pattern for both halves, which
// includes a few zero blocks for one of them and gives each half 76 of its
// 128 blocks (together the 136 nonzero ones and 16 zero ones).
template <int MP, int CT, bool TAIL, int S = 1, int TRI = 0>
__device__ __forceinline__ void chain_unit(const StageParams& prm, const ChainUnit un,
                                           unsigned char* smem_chain, int split = 0) {
  using C = ResCfg<MP, CT>;
  static_assert(C::NS == 1 || (S == 1 && !TAIL), "the split walk runs lean, one segment per wave");
  using X = float;
  using Op = typename C::Op;
  constexpr int NB = C::NB, SP = C::SP;  // NB: output pieces of 16 entries per workgroup
  constexpr int NV = MP / 16;            // pieces of a whole row
  static_assert(TRI == 0 || CT != DT_BF16, "the triangular skip is for FP32 operands");
  const int half = C::NS > 1 ? split : 0;
  Op* Ps = reinterpret_cast<Op*>(smem_chain);

  const SeqDev sq = prm.seqs[un.seq];
  const OpDev o = prm.ops[sq.op];
  const int k = prm.k;
  if (k > sq.last) return;
  if (prm.skip_kry && k < sq.kry) return;
  const bool adj = prm.adjoint != 0;
  const bool first = adj ? k == sq.last : k == 0;
  const bool final_ = adj ? k == 0 : k == sq.last;
  const bool epi = TAIL && (prm.flags & SF_EPILOGUE) && final_;
  const bool store = !epi || (prm.flags & SF_STORE_AT_EPI);


  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int j = lane & 15, g = lane >> 4;
  // 32-bit indices: the host keeps L MP 4 <= 2^31
  const int L = (int)sq.L;
  const int ncol = 1 << (k - 4);
  const int ni = (L + (1 << k) - 1) >> k;  // blocks per column
  // Blocks are numbered column by column, f = col ni + i; a segment is T
  // consecutive numbers, so it may run on into the next column (there the
  // first block has no partner in registers and loads none).
  const int nflat = ncol * ni;
  const int T = un.T;
  // per segment: first and end numbers, current block f at column fc, step fi
  int f0[S], f1[S], f[S], fc[S], fi[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    f0[q] = (un.seg0 + wave * S + q) * T;
    f1[q] = f0[q] < nflat ? (f0[q] + T < nflat ? f0[q] + T : nflat) : f0[q];
    f[q] = adj ? f1[q] - 1 : f0[q];
    fc[q] = f0[q] < nflat ? __builtin_amdgcn_readfirstlane(f[q] / ni) : 0;  // uniform
    fi[q] = f[q] - fc[q] * ni;
  }
  const int n = f1[0] - f0[0];  // the first segment is the longest (n <= 0: no work)

  // The sequence's state rows are addressed through buffer resources whose
  // range is exactly its L x MP block: the hardware range check returns zeros
  // for loads of rows outside the sequence and drops stores to them, so rows
  // l >= L and partner blocks before the start need no masking. Offsets are
  // 32-bit (the host keeps L MP 4 <= 2^31); an absent partner block is given
  // the offset 2^31, which is out of range.
  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * sizeof(X));
  const X* xin = reinterpret_cast<const X*>(first && prm.xin_first ? prm.xin_first : prm.xin) +
                 sq.x_off;
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<X*>(xin), (short)0, (int)nrec,
                                                     kBufferWord3);
  const auto rout = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<X*>(prm.xout) + sq.x_off,
                                                      (short)0, store ? (int)nrec : 0, kBufferWord3);
  const bool fin = TAIL && final_ && prm.xfinal;
  const auto rfin = __builtin_amdgcn_make_buffer_rsrc(
      fin ? reinterpret_cast<X*>(prm.xfinal) + sq.x_off : reinterpret_cast<X*>(prm.xout),
      (short)0, fin ? (int)nrec : 0, kBufferWord3);
  const uint32_t lane_off = (uint32_t)(j * MP + 4 * g) * (uint32_t)sizeof(X);
  // first time row of the block d numbers after segment q's current one (no
  // division: stepping from (fc, fi))
  auto row_at = [&](int q, int d) -> int {  // |d| <= 1
    int c = fc[q], i = fi[q] + d;
    if (i >= ni) {
      i -= ni;
      ++c;
    } else if (i < 0) {
      i += ni;
      --c;
    }
    return (i << k) + c * 16;
  };
  // byte offset of this lane's piece of block f + d (out of range outside lo..hi-1)
  auto block_off = [&](int q, int d, int lo, int hi) -> uint32_t {
    return (f[q] + d >= lo && f[q] + d < hi)
               ? lane_off + (uint32_t)row_at(q, d) * (uint32_t)(MP * sizeof(X))
               : 0x80000000u;
  };
  // stage input of this lane's row of a block, accumulator layout
  // byte offset of register piece i within a row (interleaved pairs for a split)
  auto piece = [&](int i) -> uint32_t {
    return (uint32_t)(C::NS > 1 ? 4 * ((i & 7) >> 1) + 2 * (half ^ (i >> 3)) + (i & 1) : i) * 64u;
  };
  auto load_block = [&](uint32_t off, f32x4(&v)[NV]) {
#pragma unroll
    for (int nb = 0; nb < NV; ++nb)
      v[nb] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, off + piece(nb), 0, 0));
  };
  // shifted operand for the next block: BF16 operand pieces, or FP32 as is
  constexpr int NPV = CT == DT_BF16 ? MP / 32 : NV;
  using PV = typename std::conditional<CT == DT_BF16, bf16x8, f32x4>::type;
  // (zeros when `keep` is false: the next block starts a column and has no partner)
  auto pack = [&](const f32x4(&v)[NV], bool keep, PV(&pv)[NPV]) {
    if constexpr (CT == DT_BF16) {
#pragma unroll
      for (int c = 0; c < MP / 32; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pv[c][e] = (__bf16)(keep ? v[2 * c][e] : 0.f);  // round to nearest even
          pv[c][4 + e] = (__bf16)(keep ? v[2 * c + 1][e] : 0.f);
        }
    } else {
#pragma unroll
      for (int nb = 0; nb < NV; ++nb) pv[nb] = keep ? v[nb] : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };

  const int step = adj ? -1 : 1;
  // epilogue operands: C (or Bbar^T) rows, D (or D^T), number of outputs
  const X* ecm = reinterpret_cast<const X*>(prm.small) + (adj ? o.bt : o.cout);
  const X* edm = reinterpret_cast<const X*>(prm.small) + (adj ? o.dt : o.dmat);
  const int ew = adj ? sq.p : sq.q;
  const int er = adj ? sq.q : sq.p;  // inputs of the epilogue
  // epilogue from LDS: at most 16 outputs and 16 inputs (the launch brings the LDS)
  const bool lepi = TAIL && epi && ew <= 16 && er <= 16;
  float* Cs = reinterpret_cast<float*>(smem_chain + NB * 16 * SP * sizeof(Op));
  float* Ds = Cs + 16 * C::EPS;
  // One block of segment q, its rows held in x[q]: keep the block's input as
  // the next block's shifted operand (npv), then for each group of four
  // accumulator pieces add P_k times the shifted rows, store the group and
  // load the same group of the next block into the freed registers, so that
  // the next block arrives while this one is computed. In a TAIL launch with
  // at most 16 outputs the epilogue's state part is accumulated group by group
  // too; with more outputs the epilogue takes the whole block and the next
  // block is loaded after it. The loop is unrolled by two so that the operand
  // sets swap roles without copies.
  constexpr int G = NB < 4 ? NB : 4;
  f32x4 x[S][NV];
  auto body = [&](const int q, PV(&pv)[NPV], PV(&npv)[NPV]) {
    const uint32_t off = block_off(q, 0, 0, nflat);
    const uint32_t offn = block_off(q, step, f0[q], f1[q]);  // nothing past the segment
    f32x4 ya = f32x4{0.f, 0.f, 0.f, 0.f};  // outputs of a TAIL block with at most 16 of them
    float uv[4] = {0.f, 0.f, 0.f, 0.f};   // its inputs, loaded before the next block's rows
    if constexpr (TAIL) {
      if (lepi) {
        const int64_t l = row_at(q, 0) + j;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int c = 4 * a + g;
          if (l < L && c < er)
            uv[a] = load_src<float>(prm.src, prm.src_dtype, (adj ? sq.y_off : sq.u_off) + l * er + c);
        }
      }
    }
    if constexpr (C::NS > 1) {
      // own pieces of this block's input; its other pieces are in npv already
      // (loaded there at the end of the previous block)
      const bool keep = adj ? fi[q] > 0 : fi[q] + 1 < ni;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) npv[nb] = keep ? x[q][nb] : f32x4{0.f, 0.f, 0.f, 0.f};
    } else {
      pack(x[q], adj ? fi[q] > 0 : fi[q] + 1 < ni, npv);  // partner of the next block, if any
    }
    if constexpr (CT != DT_BF16) __builtin_amdgcn_sched_barrier(0);
    // the LDS operand offset is passed through an empty asm so that the
    // compiler re-reads the power fragments each block instead of hoisting
    // them out of the loop into registers
    int lbase = j * SP + (CT == DT_BF16 ? 8 : 4) * g;
    asm volatile("" : "+v"(lbase));
#pragma unroll
    for (int n0 = 0; n0 < NB; n0 += G) {
      if constexpr (CT == DT_BF16) {  // a block without a partner gets pv = 0
        // power fragments read one MFMA step ahead of their use
        bf16x8 fa[2][G];
        auto frag = [&](int c, bf16x8(&fr)[G]) {
#pragma unroll
          for (int e = 0; e < G; ++e)
            fr[e] = *reinterpret_cast<const bf16x8*>(Ps + lbase + (n0 + e) * 16 * SP + 32 * c);
        };
        frag(0, fa[0]);
#pragma unroll
        for (int c = 0; c < MP / 32; ++c) {
          if (c + 1 < MP / 32) frag(c + 1, fa[(c + 1) & 1]);
#pragma unroll
          for (int e = 0; e < G; ++e)
            x[q][n0 + e] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[c & 1][e], pv[c], x[q][n0 + e], 0, 0, 0);
        }
      } else {
        // a lower-triangular P_k has no entries from input piece ri above
        // output piece ro (P_k^T of the adjoint none below); the test folds
        // to a constant once the loops are unrolled
        auto on = [&](int a, int nb) {
          const int ai = C::NS > 1 && a >= 8 ? ((a & 7) >> 1) : a;
          const int bi = C::NS > 1 && a >= 8 ? (nb >> 1) : nb;
          return TRI == 0 || (TRI == 1 ? ai <= bi : ai >= bi);
        };
        // power fragments of step a + 1 read while step a is contracted; the
        // scheduling fence keeps the reads from running further ahead
        f32x4 fr[2][G];
        auto frag = [&](int a, f32x4(&f)[G]) {
#pragma unroll
          for (int e = 0; e < G; ++e)
            if (on(a, n0 + e)) f[e] = *reinterpret_cast<const f32x4*>(Ps + lbase + (n0 + e) * 16 * SP + 16 * a);
        };
        frag(0, fr[0]);
#pragma unroll
        for (int a = 0; a < MP / 16; ++a) {
          if (a + 1 < MP / 16) frag(a + 1, fr[(a + 1) & 1]);
#pragma unroll
          for (int e = 0; e < G; ++e)
            if (on(a, n0 + e))
#pragma unroll
              for (int tt = 0; tt < 4; ++tt)
                x[q][n0 + e] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(fr[a & 1][e][tt], pv[a][tt], x[q][n0 + e], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int nb = n0; nb < n0 + G; ++nb) {
        const auto v = __builtin_bit_cast(u32x4, x[q][nb]);
        __builtin_amdgcn_raw_buffer_store_b128(v, rout, off + piece(nb), 0, 0);
        if constexpr (TAIL) __builtin_amdgcn_raw_buffer_store_b128(v, rfin, off + piece(nb), 0, 0);
      }
      if constexpr (TAIL) {  // up to 16 outputs: their state part group by group
        if (lepi) epi_state_lds<G>(ya, &x[q][n0], n0, Cs, C::EPS, j, g);
      }
      if (!TAIL || !epi || lepi) {  // the group's registers take the next block's rows
#pragma unroll
        for (int nb = n0; nb < n0 + G; ++nb)
          x[q][nb] = __builtin_bit_cast(
              f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, offn + piece(nb), 0, 0));
      }
      // (FP32: the loads stay behind this group's contractions, as the
      // registers they fill are only free after them)
      if constexpr (CT != DT_BF16) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (C::NS > 1) {
      // the next block's pieces of the other workgroup are only its input,
      // the shifted operand two blocks on: they go straight into this block's
      // operand registers, free now (zero, through an out-of-range offset,
      // when that block has no partner)
      const int fa = fi[q] + step, fn = fa == ni ? 0 : (fa < 0 ? ni - 1 : fa);
      const bool keepn = adj ? fn > 0 : fn + 1 < ni;
      const uint32_t offk = offn | (keepn ? 0u : 0x80000000u);
#pragma unroll
      for (int nb = NB; nb < NV; ++nb)
        pv[nb] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rin, offk + piece(nb), 0, 0));
    }
    if constexpr (TAIL) {
      // y_l = C x_l + D u_l (forward) or du_l = Bbar^T g_l + D^T dy_l (adjoint)
      const int64_t l = row_at(q, 0) + j;
      if (lepi) {
        epi_finish_lds(ya, Ds, uv, ew, er, reinterpret_cast<X*>(prm.dst), adj ? sq.u_off : sq.y_off,
                       l, l < L, j, g);
      } else if (epi) {
        res_epilogue<NB>(x[q], MP, l, l < L, ecm, edm, ew, er, prm.src,
                         prm.src_dtype, adj ? sq.y_off : sq.u_off, reinterpret_cast<X*>(prm.dst),
                         adj ? sq.u_off : sq.y_off, j, g);
        load_block(offn, x[q]);
      }
    }
    f[q] += step;
    fi[q] += step;
    if (fi[q] == ni) {
      fi[q] = 0;
      ++fc[q];
    } else if (fi[q] < 0) {
      fi[q] = ni - 1;
      --fc[q];
    }
  };

  // first loads (each segment's partner block, or zeros, and first block) go
  // out before the power is staged in LDS, so the two overlap
  PV pa[S][NPV], pb[S][NPV];
  f32x4 part[S][NV];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const bool partner = f1[q] > f0[q] && (adj ? fi[q] + 1 < ni : fi[q] > 0);
    load_block(partner ? block_off(q, -step, 0, nflat) : 0x80000000u, part[q]);
    load_block(block_off(q, 0, f0[q], f1[q]), x[q]);
  }
  // this workgroup's rows of P_k (or P_k^T) into LDS (for a split, row
  // piece e is P's piece 4 (e / 2) + 2 half + e mod 2), contraction columns
  // permuted for BF16 and for a split
  {
    const Op* P = reinterpret_cast<const Op*>(prm.P) + (adj ? o.pct : o.pc) + (int64_t)k * MP * MP;
    auto prow = [&](int r) -> int64_t {
      const int e = r >> 4;
      return (int64_t)(C::NS > 1 ? 16 * (4 * (e >> 1) + 2 * half + (e & 1)) + (r & 15) : r) * MP;
    };
    if constexpr (CT == DT_BF16) {
      for (int e = threadIdx.x; e < NB * 16 * (MP / 8); e += 512) {
        const int r = e / (MP / 8), n = (e % (MP / 8)) * 8;
        const uint4 v = *reinterpret_cast<const uint4*>(P + prow(r) + n);
        const int nb = n >> 4, g0 = (n & 15) >> 2;  // entries n..n+3 in group g0, n+4..n+7 in g0+1
        const int pos = 32 * (nb >> 1) + 8 * g0 + 4 * (nb & 1);
        *reinterpret_cast<uint2*>(Ps + r * SP + pos) = make_uint2(v.x, v.y);
        *reinterpret_cast<uint2*>(Ps + r * SP + pos + 8) = make_uint2(v.z, v.w);
      }
    } else {
      for (int e = threadIdx.x; e < NB * 16 * (MP / 4); e += 512) {
        const int r = e / (MP / 4), n = (e % (MP / 4)) * 4;
        const int ri = n >> 4;  // register piece of input piece ri (see piece())
        const int pos =
            C::NS > 1 ? 16 * ((2 * (ri >> 2) + (ri & 1)) | ((((ri >> 1) & 1) ^ half) << 3)) + (n & 15) : n;
        *reinterpret_cast<uint4*>(Ps + r * SP + pos) =
            *reinterpret_cast<const uint4*>(P + prow(r) + n);
      }
    }
    if (lepi) {  // C rows (zero beyond ew) and D (16 x 16, zero-padded)
      for (int e = threadIdx.x; e < 16 * (MP / 4); e += 512) {
        const int r = e / (MP / 4), n = (e % (MP / 4)) * 4;
        *reinterpret_cast<f32x4*>(Cs + r * C::EPS + n) =
            r < ew ? *reinterpret_cast<const f32x4*>(ecm + (int64_t)r * MP + n) : f32x4{0.f, 0.f, 0.f, 0.f};
      }
      for (int e = threadIdx.x; e < 256; e += 512) {
        const int r = e >> 4, c = e & 15;
        Ds[e] = r < ew && c < er ? edm[r * er + c] : 0.f;
      }
    }
    __syncthreads();
  }
  if (n <= 0) return;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    pack(part[q], true, pa[q]);
    if constexpr (C::NS > 1) {  // the first block's other pieces (see body)
      const bool keep = adj ? fi[q] > 0 : fi[q] + 1 < ni;
#pragma unroll
      for (int nb = NB; nb < NV; ++nb) pb[q][nb] = keep ? x[q][nb] : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
  // segments advance in lockstep; a shorter one idles once it is done
  for (int t = 0; t < n; ++t) {  // unrolled by two: the operand sets swap roles
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (t < f1[q] - f0[q]) body(q, pa[q], pb[q]);
    if (++t >= n) break;
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (t < f1[q] - f0[q]) body(q, pb[q], pa[q]);
  }
}

}  // namespace ssmc
