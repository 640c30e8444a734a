// Persistent launch of a whole ragged forward pass on the resident-power code.
//
// One workgroup per compute unit takes work items from a ticket counter in
// level order: the input pass of a sequence (its first kry stages folded, §3
// and eqs. (3.2)-(3.3)), then each later stage of it as chain units (2^k >= 16)
// or row ranges (smaller shifts). An item of level v of a sequence waits until
// every item of level v - 1 of that sequence has signalled its counter, so a
// stage only reads rows its predecessor has finished, and only overwrites the
// buffer the predecessor read once that stage is complete. A workgroup only
// ever waits for items with smaller tickets, which are held by running
// workgroups, so every wait ends and every workgroup reaches the exit.
//
// Completion: every wave drains its memory counters (its stores are in the
// L2), and after a barrier one thread issues a device-scope release fence
// (which writes this XCD's L2 back) and a relaxed device-scope increment. The
// consumer spins on relaxed device-scope loads, then takes one device-scope
// acquire fence before its workgroup reads the stage input after a barrier.
#include "stage_chain.h"

namespace ssmc {

// Segments each wave walks side by side in a chain item: about 64 registers of
// state per wave whatever the state size, so small-m items keep as many bytes
// in flight as m = 256 ones.
constexpr int persist_segments(int mp, int ct) {
  return ct == DT_BF16 ? 256 / mp : (mp == 64 ? 2 : 1);
}

int chain_segments_persist(int mp, int ct, bool tail) {
  (void)tail;
  return persist_segments(mp, ct);
}

template <int MP, int CT>
__device__ __forceinline__ void persist_item(const StageParams& base, const RItem& w, void* x0,
                                             void* x1, unsigned char* smem) {
  StageParams prm = base;
  if (w.kind == RI_INPUT) {
    prm.xin = x0;  // the input pass writes x^(kry) to x0 (kry even) or x1 (kry odd)
    prm.xout = x1;
    krylov_range<MP, CT>(prm, ResRange{w.seq, w.a, w.b, 0}, 0, smem);
    return;
  }
  prm.k = w.k;
  prm.xin = (w.k & 1) ? x1 : x0;
  prm.xout = (w.k & 1) ? x0 : x1;
  prm.skip_kry = 1;
  if (w.kind == RI_RES) {
    res_range<MP, CT>(prm, ResRange{w.seq, w.a, w.b, 0}, 0, smem);
  } else if (w.tail) {
    chain_unit<MP, CT, true, persist_segments(MP, CT)>(prm, ChainUnit{w.seq, w.a, w.b, 0}, smem);
  } else {
    chain_unit<MP, CT, false, persist_segments(MP, CT)>(prm, ChainUnit{w.seq, w.a, w.b, 0}, smem);
  }
}

template <int CT>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_persist_res(
    RPersistParams pp) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_p[];
  __shared__ int s_item, s_ok;
  int32_t* flag = pp.flag;
  for (;;) {
    __syncthreads();  // the previous item's waves are done with LDS
    if (threadIdx.x == 0) s_item = atomicAdd(pp.counters, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= pp.n_items) break;
    const RItem w = pp.items[it];
    const SeqDev sq = pp.base.seqs[w.seq];
    const int first_level = sq.kry - 1;
    const int base = pp.cnt_off[w.seq];
    if (threadIdx.x == 0) {
      bool ok = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
      if (ok && w.level > first_level) {
        // spin on relaxed device-scope loads (they bypass the caches), then one
        // acquire fence before the stage input is read
        const int c = base + (w.level - 1 - first_level);
        ok = persist_wait(pp.counters + c, pp.cnt_target[c], flag, pp.spin_limit);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_ok = ok;
    }
    __syncthreads();
    const int mp = pp.base.ops[sq.op].mp;
    if (!s_ok) {
      // a wait gave up: skip the work, still signal the item below
    } else if (mp == 64) {
      persist_item<64, CT>(pp.base, w, pp.x0, pp.x1, smem_p);
    } else if (mp == 128) {
      persist_item<128, CT>(pp.base, w, pp.x0, pp.x1, smem_p);
    } else if constexpr (CT == DT_BF16) {
      persist_item<256, CT>(pp.base, w, pp.x0, pp.x1, smem_p);
    }
    // every wave's stores have reached the L2 (all counters drained); after the
    // barrier one device-scope release writes the L2 back and publishes the item
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(pp.counters + base + (w.level - first_level), 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

size_t persist_res_lds(int ct, int max_mp) {  // with room for the tail items' C and D
  if (ct == DT_BF16) {
    if (max_mp <= 64) return ResCfg<64, DT_BF16>::LDS_TAIL;
    if (max_mp <= 128) return ResCfg<128, DT_BF16>::LDS_TAIL;
    return ResCfg<256, DT_BF16>::LDS_TAIL;
  }
  return max_mp <= 64 ? ResCfg<64, DT_F32>::LDS_TAIL : ResCfg<128, DT_F32>::LDS_TAIL;
}

template <int CT>
static hipError_t launch_pr(const RPersistParams& pp, int grid, size_t lds, hipStream_t s) {
  {
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_persist_res<CT>), lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_persist_res<CT>, dim3(grid), dim3(512), lds, s, pp);
  return hipGetLastError();
}

hipError_t launch_persist_res(int ct, const RPersistParams& pp, int grid, size_t lds, hipStream_t s) {
  if (pp.n_items <= 0 || grid <= 0) return hipSuccess;
  if (ct == DT_BF16) return launch_pr<DT_BF16>(pp, grid, lds, s);
  if (ct == DT_F32) return launch_pr<DT_F32>(pp, grid, lds, s);
  return hipErrorInvalidValue;
}

}  // namespace ssmc
