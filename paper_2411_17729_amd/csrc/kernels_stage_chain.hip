// Per-stage launch of the chain walk (one workgroup per chain unit).
#include "stage_chain.h"

namespace ssmc {

template <int MP, int CT, bool TAIL, int TRI>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_stage_chain(
    StageParams prm, const ChainUnit* units, int n_units) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_chain[];
  int u, half;
  if (!split_item<ResCfg<MP, CT>::NS>(n_units, u, half)) return;
  chain_unit<MP, CT, TAIL, 1, TRI>(prm, units[u], smem_chain, half);
}

template <int MP, int CT, bool TAIL, int TRI>
static hipError_t launch_chain_v(const StageParams& prm, const ChainUnit* units, int n_units,
                                 hipStream_t s) {
  using C = ResCfg<MP, CT>;
  constexpr size_t lds = TAIL ? C::LDS_TAIL : C::LDS;  // a tail launch stages C and D too
  {
    hipError_t e =
        ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage_chain<MP, CT, TAIL, TRI>), (size_t)((int)lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_stage_chain<MP, CT, TAIL, TRI>), dim3(split_grid(n_units, C::NS)), dim3(512), lds, s,
                     prm, units, n_units);
  return hipGetLastError();
}

template <int MP, int CT, bool TAIL>
static hipError_t launch_chain_tri(const StageParams& prm, const ChainUnit* units, int n_units, int tri,
                                   hipStream_t s) {
  if constexpr (CT == DT_BF16) {
    return launch_chain_v<MP, CT, TAIL, 0>(prm, units, n_units, s);
  } else {
    switch (tri) {
      case 1: return launch_chain_v<MP, CT, TAIL, 1>(prm, units, n_units, s);
      case 2: return launch_chain_v<MP, CT, TAIL, 2>(prm, units, n_units, s);
      default: return launch_chain_v<MP, CT, TAIL, 0>(prm, units, n_units, s);
    }
  }
}

template <int MP, int CT>
static hipError_t launch_chain_t(const StageParams& prm, const ChainUnit* units, int n_units,
                                 bool tail, int tri, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  if constexpr (ResCfg<MP, CT>::NS > 1) {
    if (tail) return hipErrorInvalidValue;  // the split walk has no tail variant
    return launch_chain_tri<MP, CT, false>(prm, units, n_units, tri, s);
  } else {
    return tail ? launch_chain_tri<MP, CT, true>(prm, units, n_units, tri, s)
                : launch_chain_tri<MP, CT, false>(prm, units, n_units, tri, s);
  }
}

bool chain_supported(int mp, int ct) {
  return (ct == DT_BF16 || ct == DT_F32) && (mp == 64 || mp == 128 || mp == 256);
}

hipError_t launch_stage_chain(int mp, int ct, const StageParams& prm, const ChainUnit* units,
                              int n_units, bool tail, int tri, hipStream_t s) {
  if (ct == DT_BF16) {
    switch (mp) {
      case 64: return launch_chain_t<64, DT_BF16>(prm, units, n_units, tail, tri, s);
      case 128: return launch_chain_t<128, DT_BF16>(prm, units, n_units, tail, tri, s);
      case 256: return launch_chain_t<256, DT_BF16>(prm, units, n_units, tail, tri, s);
    }
  } else if (ct == DT_F32) {
    switch (mp) {
      case 64: return launch_chain_t<64, DT_F32>(prm, units, n_units, tail, tri, s);
      case 128: return launch_chain_t<128, DT_F32>(prm, units, n_units, tail, tri, s);
      case 256: return launch_chain_t<256, DT_F32>(prm, units, n_units, tail, tri, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ssmc
