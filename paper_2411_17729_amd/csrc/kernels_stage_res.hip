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
// m = 256) the state rows are split between two workgroups on one XCD (split_item).
#include "stage_res.h"

namespace ssmc {

template <int MP, int CT>
__global__ __launch_bounds__(512, 1) void k_stage_res(StageParams prm, const ResRange* ranges, int n_ranges) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_res[];
  int r, half;
  if (!split_item<ResCfg<MP, CT>::NS>(n_ranges, r, half)) return;
  res_range<MP, CT>(prm, ranges[r], half, smem_res);
}

template <int MP, int CT>
static hipError_t launch_res_t(const StageParams& prm, const ResRange* ranges, int n_ranges,
                               hipStream_t s) {
  using C = ResCfg<MP, CT>;
  if (n_ranges <= 0) return hipSuccess;
  {
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage_res<MP, CT>), (size_t)((int)C::LDS));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_stage_res<MP, CT>), dim3(split_grid(n_ranges, C::NS)), dim3(512), C::LDS, s, prm,
                     ranges, n_ranges);
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
__global__ __launch_bounds__(512, 1) void k_krylov_res(StageParams prm, const ResRange* ranges, int n_ranges) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_res[];
  int r, half;
  if (!split_item<ResCfg<MP, CT>::NS>(n_ranges, r, half)) return;
  krylov_range<MP, CT>(prm, ranges[r], half, smem_res);
}

template <int MP, int CT>
static hipError_t launch_kry_t(const StageParams& prm, const ResRange* ranges, int n_ranges,
                               hipStream_t s) {
  using C = ResCfg<MP, CT>;
  if (n_ranges <= 0) return hipSuccess;
  {
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_krylov_res<MP, CT>), (size_t)((int)C::LDS));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_krylov_res<MP, CT>), dim3(split_grid(n_ranges, C::NS)), dim3(512), C::LDS, s, prm,
                     ranges, n_ranges);
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
