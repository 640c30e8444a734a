// Stage kernel with the power resident in LDS (BF16 and FP32 operands).
//
// Same stage as k_stage (§3: x_l <- x_l + P_k x_{l-2^k}, or the adjoint
// g_l <- g_l + P_k^T g_{l+2^k}), organised for HBM streaming: a workgroup
// loads its rows of P_k once into LDS (128 KB for m = 256 in BF16) and then
// its eight waves stream independent 16-row blocks of one sequence through
// the matrix cores, with no further workgroup barriers. Each wave computes
// the transposed product
//     OUT^T[n, l] = IN^T[n, l] + sum_j P[n, j] IN[l - s, j]
// so the P fragments come from LDS (A operand), the shifted rows straight
// from HBM into registers (B operand), and every lane's accumulators hold 4
// consecutive state entries of one time row: the unshifted rows are read and
// the result rows written as 16-byte vectors. When P_k does not fit (FP32,
// m = 256) the state rows are split between two workgroups (blockIdx.y).
#include "stage_res.h"

namespace ssmc {

template <int MP, int CT>
__global__ __launch_bounds__(512, 1) void k_stage_res(StageParams prm, const ResRange* ranges) {
  using C = ResCfg<MP, CT>;
  using X = float;
  using Op = typename C::Op;
  constexpr int NR = C::NR, NB = C::NB, SP = C::SP, NV = C::NV;
  static_assert(sizeof(typename C::X) == 4, "FP32 state");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_res[];
  Op* Ps = reinterpret_cast<Op*>(smem_res);

  const ResRange rg = ranges[blockIdx.x];
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
  const int n0 = blockIdx.y * NR;
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

template <int MP, int CT>
static hipError_t launch_res_t(const StageParams& prm, const ResRange* ranges, int n_ranges,
                               hipStream_t s) {
  using C = ResCfg<MP, CT>;
  if (n_ranges <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_res<MP, CT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_stage_res<MP, CT>), dim3(n_ranges, C::NS), dim3(512), C::LDS, s, prm,
                     ranges);
  return hipGetLastError();
}

bool res_supported(int mp, int ct) {
  return (ct == DT_BF16 || ct == DT_F32) && (mp == 64 || mp == 128 || mp == 256);
}

bool res_splits_rows(int mp, int ct) {
  if (ct == DT_F32 && mp == 256) return ResCfg<256, DT_F32>::NS > 1;
  return false;
}

hipError_t launch_stage_res(int mp, int ct, const StageParams& prm, const ResRange* ranges,
                            int n_ranges, hipStream_t s) {
  if (ct == DT_BF16) {
    switch (mp) {
      case 64: return launch_res_t<64, DT_BF16>(prm, ranges, n_ranges, s);
      case 128: return launch_res_t<128, DT_BF16>(prm, ranges, n_ranges, s);
      case 256: return launch_res_t<256, DT_BF16>(prm, ranges, n_ranges, s);
    }
  } else if (ct == DT_F32) {
    switch (mp) {
      case 64: return launch_res_t<64, DT_F32>(prm, ranges, n_ranges, s);
      case 128: return launch_res_t<128, DT_F32>(prm, ranges, n_ranges, s);
      case 256: return launch_res_t<256, DT_F32>(prm, ranges, n_ranges, s);
    }
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Input pass with the leading j = kry stages folded in (forward only):
//   x^(j)_l = sum_{i < 2^j} Abar^i Bbar u_{l-i} = K_j w_l,
//   w_l = [u_l; u_{l-1}; ...; u_{l-2^j+1}] (zero before the sequence start),
// with K_j resident in LDS like P_k above and w_l gathered from u.
// ---------------------------------------------------------------------------
template <int MP, int CT>
__global__ __launch_bounds__(512, 1) void k_krylov_res(StageParams prm, const ResRange* ranges) {
  using C = ResCfg<MP, CT>;
  using X = float;
  using Op = typename C::Op;
  constexpr int NR = C::NR, NB = C::NB, SP = C::SP;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_res[];
  Op* Ks = reinterpret_cast<Op*>(smem_res);

  const ResRange rg = ranges[blockIdx.x];
  const SeqDev sq = prm.seqs[rg.seq];
  const OpDev o = prm.ops[sq.op];
  if (sq.kry <= 0) return;
  const int n0 = blockIdx.y * NR;
  const int64_t L = sq.L;
  const int p = sq.p;
  const int kdim = (1 << sq.kry) * p;
  const bool final_ = sq.kry == sq.last + 1;
  const bool epi = (prm.flags & SF_EPILOGUE) && final_ && C::NS == 1;
  {
    const Op* K = reinterpret_cast<const Op*>(prm.P) + o.kc + (int64_t)n0 * MP;
    constexpr int VO = 16 / (int)sizeof(Op);
    for (int e = threadIdx.x; e < NR * (MP / VO); e += 512) {
      const int r = e / (MP / VO), c = (e % (MP / VO)) * VO;
      *reinterpret_cast<uint4*>(Ks + r * SP + c) =
          *reinterpret_cast<const uint4*>(K + (int64_t)r * MP + c);
    }
    __syncthreads();
  }
  X* xo = reinterpret_cast<X*>((sq.kry & 1) ? prm.xout : const_cast<void*>(prm.xin)) + sq.x_off;
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
    if (lv && !epi) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        *reinterpret_cast<f32x4*>(xo + l * MP + n0 + nb * 16 + 4 * g) = acc[nb];
    }
    if (epi)
      res_epilogue<NB>(acc, MP, l, lv, reinterpret_cast<const X*>(prm.small) + o.cout,
                       reinterpret_cast<const X*>(prm.small) + o.dmat, sq.q, p, usrc, udt, uoff,
                       reinterpret_cast<X*>(prm.dst), sq.y_off, j, g);
  }
}

template <int MP, int CT>
static hipError_t launch_kry_t(const StageParams& prm, const ResRange* ranges, int n_ranges,
                               hipStream_t s) {
  using C = ResCfg<MP, CT>;
  if (n_ranges <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_krylov_res<MP, CT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_krylov_res<MP, CT>), dim3(n_ranges, C::NS), dim3(512), C::LDS, s, prm,
                     ranges);
  return hipGetLastError();
}

hipError_t launch_krylov_res(int mp, int ct, const StageParams& prm, const ResRange* ranges,
                             int n_ranges, hipStream_t s) {
  if (ct == DT_BF16) {
    switch (mp) {
      case 64: return launch_kry_t<64, DT_BF16>(prm, ranges, n_ranges, s);
      case 128: return launch_kry_t<128, DT_BF16>(prm, ranges, n_ranges, s);
      case 256: return launch_kry_t<256, DT_BF16>(prm, ranges, n_ranges, s);
    }
  } else if (ct == DT_F32) {
    switch (mp) {
      case 64: return launch_kry_t<64, DT_F32>(prm, ranges, n_ranges, s);
      case 128: return launch_kry_t<128, DT_F32>(prm, ranges, n_ranges, s);
      case 256: return launch_kry_t<256, DT_F32>(prm, ranges, n_ranges, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ssmc
