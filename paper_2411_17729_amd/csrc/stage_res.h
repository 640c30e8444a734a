// Shared pieces of the stage kernels that keep the power resident in LDS.
#pragma once
#include <type_traits>

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
  // LDS rows padded by 32 bytes: 16-byte operand reads of 16 rows at a
  // stride of 512 + 16 bytes conflict two ways on gfx950, at 512 + 32 bytes not
  static constexpr int PADP = 32 / (int)sizeof(Op);
  static constexpr int SP = MP + PADP;  // LDS row stride (elements)
  static constexpr int WAVES = 8;
  static constexpr size_t LDS = (size_t)NR * SP * sizeof(Op);
  static constexpr int NV = MP / 16;  // float4 pieces of a shifted row held per lane
  // tail launches of the chain walk also stage the output matrices in LDS:
  // up to 16 rows of C (or Bbar^T) and of D (or D^T, up to 16 columns)
  static constexpr int EPS = MP + 8;  // LDS row stride of the C rows (floats, 32-byte pad)
  static constexpr size_t LDS_TAIL = LDS + (16 * EPS + 16 * 16) * sizeof(float);
};

// Workgroup -> (item, half) for launches whose items are shared by NS
// workgroups. Workgroups are dispatched to the eight XCDs in turn (workgroup b
// on XCD b mod 8), so with NS = 2 the halves of item i are workgroups
// 16 (i / 8) + i mod 8 and that + 8: both on one XCD, whose L2 serves the
// second read of the rows that both load, and dispatched together. Returns
// false for the padding workgroups past the last item.
template <int NS>
__device__ __forceinline__ bool split_item(int n, int& item, int& half) {
  static_assert(NS == 1 || NS == 2, "one or two workgroups per item");
  const int b = blockIdx.x;
  if constexpr (NS == 1) {
    item = b;
    half = 0;
  } else {
    half = (b >> 3) & 1;
    item = ((b >> 4) << 3) | (b & 7);
  }
  return item < n;
}

// workgroups of a launch of n items with NS workgroups each
inline unsigned split_grid(int n, int NS) { return NS == 1 ? (unsigned)n : 2u * (unsigned)((n + 7) & ~7); }

// Output epilogue on the matrix cores: for the lane's 16-row block,
//     Y^T[qq, l] = sum_n Cm[qq, n] X^T[n, l] + sum_c Dm[qq, c] V^T[c, l]
// (y = C x + D u forward, du = Bbar^T g + D^T dy adjoint), 16 outputs at a
// time with the FP32 16x16x4 MFMA. The state block is used where it lies:
// accumulator entry v of block nb (state index 16 nb + 4 g + v, time row j)
// is the B operand of step (nb, v), whose contraction index 4-group is g, so
// the A operand of lane (i, g) is Cm[q0 + i][16 nb + 4 g + v]. The inputs V
// enter the same accumulator, four channels per step. The result lane (j, g)
// holds outputs q0 + 4 g + v of time row l.
// Pieces of the epilogue: the state part for accumulator blocks nb0..nb0+G-1
// of outputs q0 + i (lane (i, g) supplies row i of Cm) ...
template <int G>
__device__ __forceinline__ void epi_state(f32x4& ya, const f32x4* acc, int nb0, int mp,
                                          const float* cm, int qi, bool qv, int g) {
#pragma unroll
  for (int e = 0; e < G; ++e) {
    const int nb = nb0 + e;
    const f32x4 cv = qv ? *reinterpret_cast<const f32x4*>(cm + (int64_t)qi * mp + nb * 16 + 4 * g)
                        : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) ya = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[v], acc[e][v], ya, 0, 0, 0);
  }
}
// The same two pieces with C rows and D in LDS (rows beyond w are zero) and
// the block's inputs already in registers (uv[a] = channel 4 a + g).
template <int G>
__device__ __forceinline__ void epi_state_lds(f32x4& ya, const f32x4* acc, int nb0,
                                              const float* cs, int eps, int j, int g) {
#pragma unroll
  for (int e = 0; e < G; ++e) {
    const f32x4 cv = *reinterpret_cast<const f32x4*>(cs + j * eps + (nb0 + e) * 16 + 4 * g);
#pragma unroll
    for (int v = 0; v < 4; ++v) ya = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[v], acc[e][v], ya, 0, 0, 0);
  }
}
__device__ __forceinline__ void epi_finish_lds(f32x4 ya, const float* ds, const float* uv, int w,
                                               int r_in, float* dst, int64_t dst_off, int64_t l,
                                               bool lv, int j, int g) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (4 * a >= r_in) break;
    ya = __builtin_amdgcn_mfma_f32_16x16x4f32(ds[j * 16 + 4 * a + g], uv[a], ya, 0, 0, 0);
  }
  if (lv) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int qq = 4 * g + v;
      if (qq < w) dst[dst_off + l * w + qq] = ya[v];
    }
  }
}

// ... and the input part and the store of outputs q0 + 4 g + v of time row l.
__device__ __forceinline__ void epi_finish(f32x4 ya, int q0, int qi, bool qv, const float* dm,
                                           int w, int r_in, const void* src, int sdt,
                                           int64_t src_off, float* dst, int64_t dst_off,
                                           int64_t l, bool lv, int g) {
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

template <int NB>
__device__ __forceinline__ void res_epilogue(const f32x4 (&acc)[NB], int mp, int64_t l, bool lv,
                                             const float* cm, const float* dm, int w, int r_in,
                                             const void* src, int sdt, int64_t src_off,
                                             float* dst, int64_t dst_off, int j, int g) {
  for (int q0 = 0; q0 < w; q0 += 16) {
    const int qi = q0 + j;
    const bool qv = qi < w;
    f32x4 ya = f32x4{0.f, 0.f, 0.f, 0.f};
    epi_state<NB>(ya, acc, 0, mp, cm, qi, qv, g);
    epi_finish(ya, q0, qi, qv, dm, w, r_in, src, sdt, src_off, dst, dst_off, l, lv, g);
  }
}

// One workgroup of the resident-power stage: rows rg of one sequence, state
// rows split * NR .. of the output (split > 0 only when the power is split).
template <int MP, int CT>
__device__ __forceinline__ void res_range(const StageParams& prm, const ResRange rg, int split,
                                          unsigned char* smem_res) {
  using C = ResCfg<MP, CT>;
  using X = float;
  using Op = typename C::Op;
  constexpr int NR = C::NR, NB = C::NB, SP = C::SP, NV = C::NV;
  static_assert(sizeof(typename C::X) == 4, "FP32 state");
  Op* Ps = reinterpret_cast<Op*>(smem_res);

  const SeqDev sq = prm.seqs[rg.seq];
  const OpDev o = prm.ops[sq.op];
  const int k = prm.k;
  if (k > sq.last) return;
  if (prm.skip_kry && k < sq.kry) return;
  const bool adj = prm.adjoint != 0;
  const bool first = adj ? k == sq.last : k == 0;
  const bool final_ = adj ? k == 0 : k == sq.last;
  const bool epi = (prm.flags & SF_EPILOGUE) && final_ && C::NS == 1;
  const bool store = !((prm.flags & SF_EPILOGUE) && final_) || (prm.flags & SF_STORE_AT_EPI);
  const int n0 = split * NR;
  const int64_t L = sq.L;
  const int64_t s = (int64_t)1 << k;

  // P_k (or P_k^T) rows n0..n0+NR-1 into LDS
  {
    const Op* P = reinterpret_cast<const Op*>(prm.P) + (adj ? o.pct : o.pc) + (int64_t)k * MP * MP +
                  (int64_t)n0 * MP;
    constexpr int VO = 16 / (int)sizeof(Op);
    for (int e = threadIdx.x; e < NR * (MP / VO); e += 512) {
      const int r = e / (MP / VO), c = (e % (MP / VO)) * VO;
      *reinterpret_cast<uint4*>(Ps + r * SP + c) =
          *reinterpret_cast<const uint4*>(P + (int64_t)r * MP + c);
    }
    __syncthreads();
  }

  const X* xin = reinterpret_cast<const X*>(first && prm.xin_first ? prm.xin_first : prm.xin) +
                 sq.x_off;
  X* xout = reinterpret_cast<X*>(prm.xout) + sq.x_off;
  X* xfin = final_ && prm.xfinal ? reinterpret_cast<X*>(prm.xfinal) + sq.x_off : nullptr;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int j = lane & 15, g = lane >> 4;

  const int nblk = (rg.nrows + 15) / 16;
  for (int b = wave; b < nblk; b += C::WAVES) {
    const int64_t l = (int64_t)rg.row0 + b * 16 + j;  // this lane's time row
    const bool lv = l < L && l < (int64_t)rg.row0 + rg.nrows;
    // accumulators <- unshifted row l, entries n0 + 16 nb + 4 g .. +3
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      if (lv)
        acc[nb] = *reinterpret_cast<const f32x4*>(xin + l * MP + n0 + nb * 16 + 4 * g);
      else
        acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // does any row of the block have a partner?
    const int64_t lb = (int64_t)rg.row0 + b * 16;
    const bool any = adj ? (lb + s < L) : (lb + 15 >= s);
    if (any) {
      const int64_t ls = adj ? l + s : l - s;
      const bool sv = lv && ls >= 0 && ls < L;
      const X* srow = xin + ls * MP;
      f32x4 bv[NV];
      if constexpr (CT == DT_BF16) {
        // k = 32 c + 8 g + 4 h + e for MFMA step c
#pragma unroll
        for (int c = 0; c < MP / 32; ++c)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            bv[2 * c + h] = sv ? *reinterpret_cast<const f32x4*>(srow + 32 * c + 8 * g + 4 * h)
                               : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < MP / 32; ++c) {
          bf16x8 bop;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            bop[e] = __builtin_bit_cast(__bf16, f32_to_bf16_bits(bv[2 * c][e]));
            bop[4 + e] = __builtin_bit_cast(__bf16, f32_to_bf16_bits(bv[2 * c + 1][e]));
          }
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const bf16x8 aop =
                *reinterpret_cast<const bf16x8*>(Ps + (nb * 16 + j) * SP + 32 * c + 8 * g);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[nb], 0, 0, 0);
          }
        }
      } else {
        // FP32: MFMA step (a, t) contracts k = 16 a + 4 g + t (t = 0..3)
#pragma unroll
        for (int a = 0; a < MP / 16; ++a)
          bv[a] = sv ? *reinterpret_cast<const f32x4*>(srow + 16 * a + 4 * g)
                     : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < MP / 16; ++a) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const f32x4 av =
                *reinterpret_cast<const f32x4*>(Ps + (nb * 16 + j) * SP + 16 * a + 4 * g);
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], bv[a][t], acc[nb], 0, 0, 0);
          }
        }
      }
    }
    if (lv) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if (store) *reinterpret_cast<f32x4*>(xout + l * MP + n0 + nb * 16 + 4 * g) = acc[nb];
        if (xfin) *reinterpret_cast<f32x4*>(xfin + l * MP + n0 + nb * 16 + 4 * g) = acc[nb];
      }
    }
    if (epi)  // y_l = C x_l + D u_l (forward) or du_l = Bbar^T g_l + D^T dy_l (adjoint)
      res_epilogue<NB>(acc, MP, l, lv,
                       reinterpret_cast<const X*>(prm.small) + (adj ? o.bt : o.cout),
                       reinterpret_cast<const X*>(prm.small) + (adj ? o.dt : o.dmat),
                       adj ? sq.p : sq.q, adj ? sq.q : sq.p, prm.src, prm.src_dtype,
                       adj ? sq.y_off : sq.u_off, reinterpret_cast<X*>(prm.dst),
                       adj ? sq.u_off : sq.y_off, j, g);
  }
}

// One workgroup of the input pass: rows rg of one sequence.
template <int MP, int CT>
__device__ __forceinline__ void krylov_range(const StageParams& prm, const ResRange rg, int split,
                                             unsigned char* smem_res) {
  using C = ResCfg<MP, CT>;
  using X = float;
  using Op = typename C::Op;
  constexpr int NR = C::NR, NB = C::NB, SP = C::SP;
  Op* Ks = reinterpret_cast<Op*>(smem_res);

  const SeqDev sq = prm.seqs[rg.seq];
  const OpDev o = prm.ops[sq.op];
  // x^(jj): the sequence's own input stages, or (kry_override) an earlier
  // x^(j) from the first 2^j p columns of K (K_{i+1} = [K_i | P_i K_i]),
  // written to xout and never forming y
  const int jo = prm.kry_override;
  const int jj = jo > 0 ? jo : sq.kry;
  if (jj <= 0 || jj > sq.kry || (jo > 0 && ((1 << jj) * sq.p) > MP)) return;
  const int n0 = split * NR;
  const int64_t L = sq.L;
  const int p = sq.p;
  const int kdim = (1 << jj) * p;
  const bool final_ = jo <= 0 && sq.kry == sq.last + 1;
  const bool epi = (prm.flags & SF_EPILOGUE) && final_ && C::NS == 1;
  {
    // K rows (state entries n0 ..) have stride kst >= MP; columns from kdim on
    // meet only zero window entries
    const Op* K = reinterpret_cast<const Op*>(prm.P) + o.kc + (int64_t)n0 * o.kst;
    constexpr int VO = 16 / (int)sizeof(Op);
    for (int e = threadIdx.x; e < NR * (MP / VO); e += 512) {
      const int r = e / (MP / VO), c = (e % (MP / VO)) * VO;
      *reinterpret_cast<uint4*>(Ks + r * SP + c) =
          *reinterpret_cast<const uint4*>(K + (int64_t)r * o.kst + c);
    }
    __syncthreads();
  }
  X* xo = reinterpret_cast<X*>(jo > 0 ? prm.xout
                                      : (sq.kry & 1) ? prm.xout : const_cast<void*>(prm.xin)) + sq.x_off;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int j = lane & 15, g = lane >> 4;
  // Window column kk of row l is u[l - kk / p][kk % p] (zero before the start).
  // A lane's columns come in runs of 8 (BF16) or 4 (FP32) consecutive kk;
  // each run is walked with one division and then a carried (lag, channel).
  const void* usrc = prm.src;
  const int udt = prm.src_dtype;
  const int64_t uoff = sq.u_off;
  // FP32 input with 4 | p and 16-byte aligned rows: the runs split into
  // 16-byte pieces of one input row each.
  const bool vec4 = udt == DT_F32 && (p & 3) == 0 && (uoff & 3) == 0 &&
                    (reinterpret_cast<uintptr_t>(usrc) & 15) == 0;
  auto run = [&](int64_t l, int kk0, float* dstv, int n) {
    int lag = kk0 / p, ch = kk0 - lag * p;
    if (vec4) {
      for (int e = 0; e < n; e += 4) {
        const int64_t lu = l - lag;
        const f32x4 v = (kk0 + e < kdim && lu >= 0)
                            ? *reinterpret_cast<const f32x4*>(
                                  reinterpret_cast<const float*>(usrc) + uoff + lu * p + ch)
                            : f32x4{0.f, 0.f, 0.f, 0.f};
        dstv[e] = v[0];
        dstv[e + 1] = v[1];
        dstv[e + 2] = v[2];
        dstv[e + 3] = v[3];
        ch += 4;
        if (ch == p) {
          ch = 0;
          ++lag;
        }
      }
      return;
    }
    for (int e = 0; e < n; ++e) {
      const int64_t lu = l - lag;
      dstv[e] = (kk0 + e < kdim && lu >= 0) ? load_src<X>(usrc, udt, uoff + lu * p + ch) : 0.f;
      if (++ch == p) {
        ch = 0;
        ++lag;
      }
    }
  };
  const int nblk = (rg.nrows + 15) / 16;
  X* dst = reinterpret_cast<X*>(prm.dst);
  const X* cm = reinterpret_cast<const X*>(prm.small) + o.cout;
  const X* dm = reinterpret_cast<const X*>(prm.small) + o.dmat;
  if (vec4 && L * p * 4 <= ((int64_t)1 << 31)) {
    // Fast path: a block's whole window is fetched with one 16-byte load per
    // piece (a lane's pieces are fixed offsets from its row's start, so they
    // are computed once), through a buffer resource over the sequence's u:
    // rows before the start fall outside its range and read as zeros. The
    // next block's window is loaded while the current one is computed.
    constexpr int NW = MP / 16;  // 16-byte pieces per lane and block
    int32_t koff[NW];
    bool kval[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int kk0 = CT == DT_BF16 ? 32 * (w >> 1) + 8 * g + 4 * (w & 1) : 16 * w + 4 * g;
      const int lag = kk0 / p, ch = kk0 - lag * p;
      kval[w] = kk0 < kdim;
      koff[w] = (ch - lag * p) * 4;
    }
    const auto ru = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(reinterpret_cast<const float*>(usrc) + uoff), (short)0,
        (int)(uint32_t)(L * p * 4), kBufferWord3);
    auto gather = [&](int b, f32x4(&wv)[NW]) {
      const uint32_t base = (uint32_t)(((int64_t)rg.row0 + b * 16 + j) * p * 4);
#pragma unroll
      for (int w = 0; w < NW; ++w)
        wv[w] = __builtin_bit_cast(
            f32x4, __builtin_amdgcn_raw_buffer_load_b128(ru, kval[w] ? base + koff[w] : 0x80000000u, 0, 0));
    };
    // one block from its window: BF16 operands (already converted) or FP32 pieces
    using WOP = typename std::conditional<CT == DT_BF16, bf16x8, f32x4>::type;
    constexpr int NO = CT == DT_BF16 ? MP / 32 : MP / 16;
    auto block = [&](int b, const WOP(&wo)[NO]) {
      const int64_t l = (int64_t)rg.row0 + b * 16 + j;
      const bool lv = l < L && l < (int64_t)rg.row0 + rg.nrows;
      f32x4 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      // the LDS offset goes through an empty asm so that the K fragments are
      // read per block rather than hoisted out of the block loop into registers
      int lbase = j * SP + (CT == DT_BF16 ? 8 : 4) * g;
      asm volatile("" : "+v"(lbase));
      if constexpr (CT == DT_BF16) {
#pragma unroll
        for (int c = 0; c < MP / 32; ++c) {
          if (32 * c >= kdim) break;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const bf16x8 aop = *reinterpret_cast<const bf16x8*>(Ks + lbase + nb * 16 * SP + 32 * c);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, wo[c], acc[nb], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < MP / 16; ++a) {
          if (16 * a >= kdim) break;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const f32x4 av = *reinterpret_cast<const f32x4*>(Ks + lbase + nb * 16 * SP + 16 * a);
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], wo[a][t], acc[nb], 0, 0, 0);
          }
        }
      }
      if (lv && (!epi || (prm.flags & SF_STORE_AT_EPI))) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          *reinterpret_cast<f32x4*>(xo + l * MP + n0 + nb * 16 + 4 * g) = acc[nb];
      }
      if (epi) res_epilogue<NB>(acc, MP, l, lv, cm, dm, sq.q, p, usrc, udt, uoff, dst, sq.y_off, j, g);
    };
    f32x4 wv[NW];
    int b = wave;
    if (b < nblk) gather(b, wv);
    for (; b < nblk; b += C::WAVES) {
      // take this block's window out of wv, then reuse wv for the next block's loads
      WOP wo[NO];
      if constexpr (CT == DT_BF16) {
#pragma unroll
        for (int c = 0; c < NO; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            wo[c][e] = (__bf16)wv[2 * c][e];  // round to nearest even
            wo[c][4 + e] = (__bf16)wv[2 * c + 1][e];
          }
      } else {
#pragma unroll
        for (int a = 0; a < NO; ++a) wo[a] = wv[a];
      }
      if (b + C::WAVES < nblk) gather(b + C::WAVES, wv);
      block(b, wo);
    }
    return;
  }
  for (int b = wave; b < nblk; b += C::WAVES) {
    const int64_t l = (int64_t)rg.row0 + b * 16 + j;
    const bool lv = l < L && l < (int64_t)rg.row0 + rg.nrows;
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (CT == DT_BF16) {
      for (int c = 0; c < (kdim + 31) / 32; ++c) {
        float wvals[8];
        if (lv)
          run(l, 32 * c + 8 * g, wvals, 8);
        else
          for (int e = 0; e < 8; ++e) wvals[e] = 0.f;
        bf16x8 bop;
#pragma unroll
        for (int e = 0; e < 8; ++e) bop[e] = __builtin_bit_cast(__bf16, f32_to_bf16_bits(wvals[e]));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf16x8 aop =
              *reinterpret_cast<const bf16x8*>(Ks + (nb * 16 + j) * SP + 32 * c + 8 * g);
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[nb], 0, 0, 0);
        }
      }
    } else {
      for (int a = 0; a < (kdim + 15) / 16; ++a) {
        float wvals[4];
        if (lv)
          run(l, 16 * a + 4 * g, wvals, 4);
        else
          for (int t = 0; t < 4; ++t) wvals[t] = 0.f;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const f32x4 av =
              *reinterpret_cast<const f32x4*>(Ks + (nb * 16 + j) * SP + 16 * a + 4 * g);
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], wvals[t], acc[nb], 0, 0, 0);
        }
      }
    }
    if (lv && (!epi || (prm.flags & SF_STORE_AT_EPI))) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        *reinterpret_cast<f32x4*>(xo + l * MP + n0 + nb * 16 + 4 * g) = acc[nb];
    }
    if (epi) res_epilogue<NB>(acc, MP, l, lv, cm, dm, sq.q, p, usrc, udt, uoff, dst, sq.y_off, j, g);
  }
}

}  // namespace ssmc
