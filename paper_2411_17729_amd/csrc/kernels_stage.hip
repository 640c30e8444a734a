// Stage kernel of the fast cascade (§3 of Beylkin, arXiv 2411.17729).
//
// One launch applies stage k to every row tile of every sequence:
//   forward  (eqs. (3.2)-(3.4), general step):  x_l <- x_l + P_k x_{l-2^k},   2^k <= l < L
//   adjoint  (transpose, reversed shift):        g_l <- g_l + P_k^T g_{l+2^k}, l + 2^k < L
// with P_k = Abar^(2^k). Rows without a partner are copied. The state is
// stored time-major (L x mp per sequence), so a time shift is a row offset
// and each row tile is a dense GEMM  OUT[tile] = IN[tile] + IN[tile - s] * P_k^T
// of shape BM x mp x mp. The unshifted rows initialise the MFMA accumulators,
// so the stage's addition is the accumulate of the matrix cores.
//
// The input rows of the first stage come from a projection pass (k_project:
// v_l = Bbar u_l forward, g_l = C^T dy_l adjoint); at the last stage the
// output rows are written instead of (or besides) the state
// (y_l = C x_l + D u_l forward, du_l = Bbar^T g_l + D^T dy_l adjoint).
#include <type_traits>

#include "stage_common.h"

namespace ssmc {

template <int MP, int CT, int BM_ = stage_bm(MP, CT)>
struct StageCfg {
  using TR = CTraits<CT>;
  using X = typename TR::X;
  using Op = typename TR::Op;
  static constexpr int WC = MP >= 64 ? 4 : 2;  // waves across the state columns
  static constexpr int WR = 4 / WC;            // waves across the rows
  static constexpr int CW = MP / WC;           // columns per wave
  static constexpr int CB = CW / 16;           // 16-column blocks per wave
  static constexpr int BM = BM_;               // rows per tile
  static constexpr int RB = BM / (WR * 16);    // 16-row blocks per wave
  static constexpr int KC0 = 128 / (int)sizeof(Op);
  static constexpr int KC = KC0 < MP ? KC0 : MP;  // K chunk staged in LDS
  static constexpr int NCH = MP / KC;
  static constexpr int KSTEPS = KC / TR::KI;
  static constexpr int SA = KC + TR::PAD;  // LDS row stride (elements)
  static constexpr int SE = MP + 1;        // epilogue row stride
  static constexpr size_t LDS_MM = (size_t)(BM + MP) * SA * sizeof(Op);
  static constexpr size_t LDS_EPI = (size_t)WR * 16 * SE * sizeof(X);
  static constexpr size_t LDS = LDS_MM > LDS_EPI ? LDS_MM : LDS_EPI;
  static_assert(RB >= 1 && RB * WR * 16 == BM, "tile rows");
  static_assert(KSTEPS >= 1 && NCH * KC == MP, "K chunking");
  static_assert((SA * sizeof(Op)) % 16 == 0, "LDS rows must stay 16-byte aligned");
};

// One row tile of one stage (the body shared by the per-stage kernel and the
// persistent ragged kernel). smem must hold StageCfg<MP, CT>::LDS bytes.
template <int MP, int CT, int BM_ = stage_bm(MP, CT)>
__device__ __forceinline__ void stage_tile(const StageParams& prm, const Tile t,
                                           unsigned char* smem) {
  using C = StageCfg<MP, CT, BM_>;
  using X = typename C::X;
  using Op = typename C::Op;
  using TR = typename C::TR;
  using Acc = typename TR::Acc;
  constexpr int BM = C::BM, RB = C::RB, CB = C::CB, CW = C::CW, WC = C::WC, WR = C::WR;
  constexpr int KC = C::KC, SA = C::SA, SE = C::SE;

  Op* As = reinterpret_cast<Op*>(smem);
  Op* Bs = As + BM * SA;
  X* Es = reinterpret_cast<X*>(smem);

  const SeqDev sq = prm.seqs[t.seq];
  const OpDev o = prm.ops[sq.op];

  const bool noupd = (prm.flags & SF_NOUPDATE) != 0;
  const int k = prm.k;
  if (!noupd && k > sq.last) return;
  if (!noupd && prm.skip_kry && k < sq.kry) return;
  const bool adj = prm.adjoint != 0;
  const bool first = !noupd && (adj ? k == sq.last : k == 0);
  const bool final_ = noupd || (adj ? k == 0 : k == sq.last);
  const bool epi = (prm.flags & SF_EPILOGUE) && final_;
  const bool store = !epi || (prm.flags & SF_STORE_AT_EPI);

  const int64_t L = sq.L;
  const int64_t row0 = t.row0;
  const int64_t s = noupd ? 0 : ((int64_t)1 << k);
  const int64_t rlast = (row0 + BM < L ? row0 + BM : L) - 1;
  const bool upd = !noupd && (adj ? (row0 + s < L) : (rlast >= s));

  const X* small = reinterpret_cast<const X*>(prm.small);
  const X* xin = reinterpret_cast<const X*>(first && prm.xin_first ? prm.xin_first : prm.xin) +
                 sq.x_off;
  X* xout = reinterpret_cast<X*>(prm.xout) + sq.x_off;
  const int r_in = adj ? sq.q : sq.p;  // width of the src rows
  const int64_t src_off = adj ? sq.y_off : sq.u_off;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int lrow = lane & 15, lgrp = lane >> 4;

  // ---- accumulators <- unshifted rows ----
  Acc acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int col = wc * CW + cb * 16 + lrow;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t l = row0 + (wr * RB + rb) * 16 + TR::acc_row(lgrp, v);
        acc[rb][cb][v] = l < L ? xin[l * MP + col] : (X)0;
      }
    }
  }

  // ---- shifted rows times P_k^T (or P_k for the adjoint) on MFMA ----
  // K is staged through LDS in chunks; the global loads of chunk ch+1 are
  // issued into registers before the MFMAs of chunk ch.
  if (upd) {
    const Op* P = reinterpret_cast<const Op*>(prm.P) + (adj ? o.pct : o.pc) + (int64_t)k * MP * MP;
    constexpr int VX = 16 / (int)sizeof(X);  // state elements per 16-byte load
    constexpr int GA = KC / VX;              // 16-byte groups per A row chunk
    constexpr int VO = 16 / (int)sizeof(Op);
    constexpr int GB = KC / VO;
    constexpr int NA = (BM * GA + 255) / 256;  // A groups per thread
    constexpr int NB = (MP * GB + 255) / 256;  // B groups per thread
    using XV = typename std::conditional<sizeof(X) == 4, float4, double2>::type;
    XV ra[NA];
    // X rows of chunk ch (HBM) into registers
    auto fetch = [&](int ch) {
      const int k0 = ch * KC;
#pragma unroll
      for (int it = 0; it < NA; ++it) {
        const int g = tid + it * 256;
        const int i = g / GA, kk = (g % GA) * VX;
        const int64_t l = row0 + i;
        const int64_t ls = adj ? l + s : l - s;
        if (g < BM * GA && l < L && ls >= 0 && ls < L)
          ra[it] = *reinterpret_cast<const XV*>(xin + ls * MP + k0 + kk);
        else
          ra[it] = XV{};
      }
    };
    // registers -> A chunk (converted to the operand type); P_k chunk (L2) -> LDS
    auto stash = [&](int ch) {
      const int k0 = ch * KC;
#pragma unroll
      for (int it = 0; it < NA; ++it) {
        const int g = tid + it * 256;
        if (g < BM * GA) {
          const int i = g / GA, kk = (g % GA) * VX;
          Op* d = As + i * SA + kk;
          const X* vals = reinterpret_cast<const X*>(&ra[it]);
#pragma unroll
          for (int e = 0; e < VX; ++e) d[e] = to_op<Op, X>(vals[e]);
        }
      }
#pragma unroll
      for (int it = 0; it < NB; ++it) {
        const int g = tid + it * 256;
        if (g < MP * GB) {
          const int n = g / GB, kk = (g % GB) * VO;
          *reinterpret_cast<uint4*>(Bs + n * SA + kk) =
              *reinterpret_cast<const uint4*>(P + (int64_t)n * MP + k0 + kk);
        }
      }
    };
    fetch(0);
    for (int ch = 0; ch < C::NCH; ++ch) {
      __syncthreads();
      stash(ch);
      __syncthreads();
      if (ch + 1 < C::NCH) fetch(ch + 1);
#pragma unroll
      for (int ks = 0; ks < C::KSTEPS; ++ks) {
        const int kof = ks * TR::KI + lgrp * TR::KPL;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const Op* ap = As + ((wr * RB + rb) * 16 + lrow) * SA + kof;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const Op* bp = Bs + (wc * CW + cb * 16 + lrow) * SA + kof;
            acc[rb][cb] = Mfma<CT>::run(ap, bp, acc[rb][cb]);
          }
        }
      }
    }
  }

  // ---- store the state rows ----
  X* xfin = final_ && prm.xfinal ? reinterpret_cast<X*>(prm.xfinal) + sq.x_off : nullptr;
  if (store || xfin) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int col = wc * CW + cb * 16 + lrow;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t l = row0 + (wr * RB + rb) * 16 + TR::acc_row(lgrp, v);
          if (l < L) {
            if (store) xout[l * MP + col] = acc[rb][cb][v];
            if (xfin) xfin[l * MP + col] = acc[rb][cb][v];
          }
        }
      }
    }
  }

  // ---- output projection ----
  if (epi) {
    const int w = adj ? sq.p : sq.q;
    const X* cm = small + (adj ? o.bt : o.cout);  // w x MP
    const X* dm = small + (adj ? o.dt : o.dmat);  // w x r_in
    const int64_t dst_off = adj ? sq.u_off : sq.y_off;
    X* dst = reinterpret_cast<X*>(prm.dst);
    for (int rb = 0; rb < RB; ++rb) {
      __syncthreads();
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int col = wc * CW + cb * 16 + lrow;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Es[(wr * 16 + TR::acc_row(lgrp, v)) * SE + col] = acc[rb][cb][v];
        }
      }
      __syncthreads();
      for (int oi = tid; oi < WR * 16 * w; oi += 256) {
        const int er = oi / w, j = oi % w;
        const int64_t l = row0 + ((er / 16) * RB + rb) * 16 + (er % 16);
        if (l < L) {
          X a0 = 0, a1 = 0;
          const X* crow = cm + (int64_t)j * MP;
          const X* erow = Es + er * SE;
          for (int n = 0; n < MP; n += 2) {
            a0 += crow[n] * erow[n];
            a1 += crow[n + 1] * erow[n + 1];
          }
          X val = a0 + a1;
          for (int jj = 0; jj < r_in; ++jj)
            val += dm[j * r_in + jj] * load_src<X>(prm.src, prm.src_dtype, src_off + l * r_in + jj);
          dst[dst_off + l * w + j] = val;
        }
      }
    }
  }
}


// Consecutive tiles to one XCD: hardware hands workgroups to the 8 XCDs
// round-robin, so tile t of XCD x is start_x + blockIdx.x / 8.
__device__ __forceinline__ int xcd_tile(int nt) {
  const int b = blockIdx.x;
  const int xcd = b & 7, per = nt >> 3, rem = nt & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + (b >> 3);
}

template <int MP, int CT, int BM>
__global__ __launch_bounds__(256, 2) void k_stage(StageParams prm) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[StageCfg<MP, CT, BM>::LDS];
  stage_tile<MP, CT, BM>(prm, prm.tiles[xcd_tile(prm.n_tiles)], smem);
}

// ---------------------------------------------------------------------------
// Input projection of a row tile: out_l = M src_l for every row l of the tile,
//   forward: v_l = Bbar u_l   (M = Bbar, MP x p; the columns of V^(0), §3)
//   adjoint: g_l = C^T dy_l   (M = C^T,  MP x q)
// One workgroup per tile; M and the tile's source rows are staged in LDS in
// chunks of 32 source columns; thread t owns state column t % MP.
// ---------------------------------------------------------------------------
template <int MP, typename X>
struct ProjCfg {
  static constexpr int PB = 64;  // rows per sub-block
  static constexpr int RCH = 32; // source columns per LDS chunk
  static constexpr size_t LDS = (size_t)(MP + PB) * (RCH + 1) * sizeof(X);
};

// rows: the tile height of the launch's tile table.
template <int MP, typename X>
__device__ __forceinline__ void project_tile(const StageParams& prm, const Tile t, int rows,
                                             unsigned char* smem) {
  constexpr int PB = ProjCfg<MP, X>::PB;
  constexpr int RCH = ProjCfg<MP, X>::RCH;
  constexpr int RG = 256 / MP;     // row groups
  constexpr int RPT = PB / RG;     // rows per thread per sub-block
  X (*Ms)[RCH + 1] = reinterpret_cast<X (*)[RCH + 1]>(smem);
  X (*Us)[RCH + 1] = reinterpret_cast<X (*)[RCH + 1]>(smem + (size_t)MP * (RCH + 1) * sizeof(X));
  const SeqDev sq = prm.seqs[t.seq];
  const OpDev o = prm.ops[sq.op];
  const bool adj = prm.adjoint != 0;
  const int r = adj ? sq.q : sq.p;
  const int64_t src_off = adj ? sq.y_off : sq.u_off;
  const X* M = reinterpret_cast<const X*>(prm.small) + (adj ? o.ct : o.bin);
  X* out = reinterpret_cast<X*>(prm.xout) + sq.x_off;
  // rows of this tile: [t.row0, min(L, t.row0 + rows))
  const int64_t L = (int64_t)t.row0 + rows < sq.L ? (int64_t)t.row0 + rows : sq.L;
  const int tid = threadIdx.x, n = tid % MP, rg = tid / MP;
  for (int sb = 0; sb < rows; sb += PB) {
    const int64_t row0 = (int64_t)t.row0 + sb;
    if (row0 >= L) break;
    X acc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) acc[i] = 0;
    for (int j0 = 0; j0 < r; j0 += RCH) {
      const int jn = r - j0 < RCH ? r - j0 : RCH;
      __syncthreads();
      for (int e = tid; e < MP * RCH; e += 256) {
        const int nn = e / RCH, jj = e % RCH;
        Ms[nn][jj] = jj < jn ? M[nn * r + j0 + jj] : (X)0;
      }
      for (int e = tid; e < PB * RCH; e += 256) {
        const int i = e / RCH, jj = e % RCH;
        const int64_t l = row0 + i;
        Us[i][jj] = (jj < jn && l < L) ? load_src<X>(prm.src, prm.src_dtype, src_off + l * r + j0 + jj)
                                       : (X)0;
      }
      __syncthreads();
      for (int jj = 0; jj < jn; ++jj) {
        const X mv = Ms[n][jj];
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc[i] += mv * Us[i * RG + rg][jj];
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t l = row0 + i * RG + rg;
      if (l < L) out[l * MP + n] = acc[i];
    }
  }
}

template <int MP, typename X>
__global__ __launch_bounds__(256) void k_project(StageParams prm, int rows) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[ProjCfg<MP, X>::LDS];
  project_tile<MP, X>(prm, prm.tiles[xcd_tile(prm.n_tiles)], rows, smem);
}

// ---------------------------------------------------------------------------
// Persistent ragged forward pass: one launch works through all items of the
// plan (projection tiles, then stage 0 tiles, stage 1 tiles, ... of every
// sequence) from a ticket counter. A stage-k tile of a sequence starts when
// all stage-(k-1) tiles of that sequence are done (a completion counter per
// sequence and stage). Dependencies always hold smaller tickets, and a
// workgroup only waits after taking its ticket, so the smallest unfinished
// ticket can always proceed: there is no deadlock for any grid size, and
// every workgroup leaves once the counter passes the last item.
// ---------------------------------------------------------------------------
template <int CT>
struct PersistLds {
  using X = typename CTraits<CT>::X;
  static constexpr size_t m1(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t S = m1(m1(StageCfg<32, CT>::LDS, StageCfg<64, CT>::LDS),
                                 m1(StageCfg<128, CT>::LDS, StageCfg<256, CT>::LDS));
  static constexpr size_t Pj = m1(m1(ProjCfg<32, X>::LDS, ProjCfg<64, X>::LDS),
                                  m1(ProjCfg<128, X>::LDS, ProjCfg<256, X>::LDS));
  static constexpr size_t LDS = m1(S, Pj);
};

template <int CT>
__global__ __launch_bounds__(256, 1) void k_persistent(PersistParams pp) {
  using X = typename CTraits<CT>::X;
  __shared__ __attribute__((aligned(16))) unsigned char smem[PersistLds<CT>::LDS];
  __shared__ int s_item, s_ok;
  int32_t* flag = pp.flag;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(pp.counters, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= pp.n_items) break;
    const PItem w = pp.items[it];
    if (threadIdx.x == 0) {
      bool ok = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
      if (ok && w.k >= 0) {
        // relaxed device-scope spin (bypasses the caches), then one acquire fence
        const int32_t* c = pp.counters + pp.cnt_off[w.seq] + w.k;  // level k-1
        ok = persist_wait(c, pp.ntiles[w.seq], flag, pp.spin_limit);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_ok = ok;
    }
    __syncthreads();
    StageParams prm = pp.base;
    const Tile t{w.seq, w.row0};
    if (!s_ok) {
      // a wait gave up: skip the work, still signal the item below
    } else if (w.k < 0) {
      prm.xout = pp.x0;
      switch (w.mp) {
        case 32: project_tile<32, X>(prm, t, stage_bm(32, CT), smem); break;
        case 64: project_tile<64, X>(prm, t, stage_bm(64, CT), smem); break;
        case 128: project_tile<128, X>(prm, t, stage_bm(128, CT), smem); break;
        default: project_tile<256, X>(prm, t, stage_bm(256, CT), smem); break;
      }
    } else {
      prm.k = w.k;
      prm.xin = (w.k & 1) ? pp.x1 : pp.x0;
      prm.xout = (w.k & 1) ? pp.x0 : pp.x1;
      switch (w.mp) {
        case 32: stage_tile<32, CT>(prm, t, smem); break;
        case 64: stage_tile<64, CT>(prm, t, smem); break;
        case 128: stage_tile<128, CT>(prm, t, smem); break;
        default: stage_tile<256, CT>(prm, t, smem); break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this item's rows, visible device-wide
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(pp.counters + pp.cnt_off[w.seq] + w.k + 1, 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_persistent(int ct, const PersistParams& pp, int grid, hipStream_t s) {
  if (pp.n_items <= 0 || grid <= 0) return hipSuccess;
  switch (ct) {
    case DT_BF16: hipLaunchKernelGGL(k_persistent<DT_BF16>, dim3(grid), dim3(256), 0, s, pp); break;
    case DT_F32: hipLaunchKernelGGL(k_persistent<DT_F32>, dim3(grid), dim3(256), 0, s, pp); break;
    case DT_F64: hipLaunchKernelGGL(k_persistent<DT_F64>, dim3(grid), dim3(256), 0, s, pp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int persistent_blocks_per_cu(int ct) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (ct) {
    case DT_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<DT_BF16>, 256, 0); break;
    case DT_F32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<DT_F32>, 256, 0); break;
    case DT_F64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<DT_F64>, 256, 0); break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <int MP, typename X>
static hipError_t launch_proj(const StageParams& prm, int rows, hipStream_t s) {
  if (prm.n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_project<MP, X>), dim3(prm.n_tiles), dim3(256), 0, s, prm, rows);
  return hipGetLastError();
}

hipError_t launch_project(int mp, int state_f64, int rows, const StageParams& prm,
                          hipStream_t s) {
  if (rows <= 0) return hipErrorInvalidValue;
  switch (mp) {
    case 32: return state_f64 ? launch_proj<32, double>(prm, rows, s) : launch_proj<32, float>(prm, rows, s);
    case 64: return state_f64 ? launch_proj<64, double>(prm, rows, s) : launch_proj<64, float>(prm, rows, s);
    case 128: return state_f64 ? launch_proj<128, double>(prm, rows, s) : launch_proj<128, float>(prm, rows, s);
    case 256: return state_f64 ? launch_proj<256, double>(prm, rows, s) : launch_proj<256, float>(prm, rows, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MP, int CT, int BM>
static hipError_t launch_one(const StageParams& prm, hipStream_t s) {
  if (prm.n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_stage<MP, CT, BM>), dim3(prm.n_tiles), dim3(256), 0, s, prm);
  return hipGetLastError();
}

template <int MP, int CT>
static hipError_t launch_bm(int bm, const StageParams& prm, hipStream_t s) {
  constexpr int D = stage_bm(MP, CT);
  if (bm == D) return launch_one<MP, CT, D>(prm, s);
  if (bm == D / 2) return launch_one<MP, CT, D / 2>(prm, s);
  return hipErrorInvalidValue;
}

template <int CT>
static hipError_t launch_ct(int mp, int bm, const StageParams& prm, hipStream_t s) {
  switch (mp) {
    case 32: return launch_bm<32, CT>(bm, prm, s);
    case 64: return launch_bm<64, CT>(bm, prm, s);
    case 128: return launch_bm<128, CT>(bm, prm, s);
    case 256: return launch_bm<256, CT>(bm, prm, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage(int mp, int ct, int bm, const StageParams& prm, hipStream_t s) {
  switch (ct) {
    case DT_BF16: return launch_ct<DT_BF16>(mp, bm, prm, s);
    case DT_F32: return launch_ct<DT_F32>(mp, bm, prm, s);
    case DT_F64: return launch_ct<DT_F64>(mp, bm, prm, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssmc
