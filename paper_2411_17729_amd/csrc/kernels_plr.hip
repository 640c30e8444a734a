// Partitioned low-rank (PLR) powers, §5: the off-diagonal blocks of the
// dyadic partition of P_k = Abar^(2^k) kept in low-rank form, built on the GPU
// at prepare time from the FP64 powers, and the stage x_l += P~_k x_{l-2^k}
// applied in that form on the matrix cores.
//
// Record of one operator and stage (compute type, zero padded): for levels
// d = 1..D (block size s = mp >> d) and nodes g < 2^(d-1), the lower block
// (side 0: rows [2gs + s, 2gs + 2s) x columns [2gs, 2gs + s)) and the upper
// block (side 1, the transposed position), each as U' (s x kPlrRC) followed
// by V^T (kPlrRC x s); then the mp/16 dense diagonal leaves (16 x 16, row
// major). Within every 16 columns of U' the ranks are stored in the order the
// stage kernel's lanes read them: U'[i][16b + 4a + v] = U[i][16b + a + 4v].
// The ranks of a record sit in a table of 32 entries per record.
#include "plr.h"
#include "stage_common.h"

namespace ssmc {

namespace {

constexpr int kPlrThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pivoted Gram-Schmidt of one off-diagonal block B (s x s, s <= 128): columns
// of Q chosen greedily by the largest residual column norm, each
// re-orthogonalized against the earlier ones, until the residual B - Q Q^T B
// has Frobenius norm <= tol; then V^T = Q^T B from the original block. The
// block, its residual and the column norms live in LDS; Q (FP64) in `qs`.
// A rank above kPlrRC is recorded as kPlrRC + 1 with zero factors. A job with
// d == 0 copies the dense diagonal leaves instead.
template <typename CT>
__global__ __launch_bounds__(kPlrThreads) void k_plr_compress(PlrCompressParams prm) {
  extern __shared__ double lds[];
  const PlrJob jb = prm.jobs[blockIdx.x];
  const OpDev& o = prm.ops[jb.op];
  const int mp = o.mp, t = threadIdx.x;
  const double* Pk = prm.pw + o.pw + (int64_t)jb.k * mp * mp;
  CT* rec = reinterpret_cast<CT*>(prm.rec) + prm.rec_off[jb.op] + (int64_t)jb.k * plr_rec_elems(mp);
  if (jb.d == 0) {
    CT* lv = rec + plr_leaf_off(mp);
    for (int e = t; e < mp * kPlrLeaf; e += kPlrThreads) {
      const int f = e / (kPlrLeaf * kPlrLeaf), w = e % (kPlrLeaf * kPlrLeaf);
      const int i = f * kPlrLeaf + w / kPlrLeaf, j = f * kPlrLeaf + w % kPlrLeaf;
      lv[e] = (CT)Pk[(int64_t)i * mp + j];
    }
    return;
  }
  const int s = mp >> jb.d, a = 2 * jb.g * s;
  const int row0 = jb.side == 0 ? a + s : a, col0 = jb.side == 0 ? a : a + s;
  const int ld = s + 1;  // padded column stride: column-owning threads hit distinct banks
  double* R = lds;                   // R[j * ld + i], column j of the residual
  double* cn = R + s * ld;           // residual column norms
  double* q = cn + s;                // current basis vector
  double* h = q + s;                 // its projections on the earlier ones
  double* misc = h + kPlrRC;         // [0] total, [1] |q|^2, [2] pivot (as double)
  double* Q = prm.qs + (int64_t)blockIdx.x * kPlrRC * kPlrMaxS;  // Q[c * s + i]

  for (int e = t; e < s * s; e += kPlrThreads) {
    const int i = e / s, j = e % s;
    R[j * ld + i] = Pk[(int64_t)(row0 + i) * mp + col0 + j];
  }
  __syncthreads();
  int r = 0;
  for (;;) {
    if (t < s) {
      double acc = 0.0;
      for (int i = 0; i < s; ++i) acc += R[t * ld + i] * R[t * ld + i];
      cn[t] = acc;
    }
    __syncthreads();
    if (t < 64) {
      double tot = 0.0, best = -1.0;
      int bj = 0;
      for (int j = t; j < s; j += 64) {
        tot += cn[j];
        if (cn[j] > best) {
          best = cn[j];
          bj = j;
        }
      }
      tot = wave_sum(tot);
#pragma unroll
      for (int o2 = 32; o2 > 0; o2 >>= 1) {
        const double ob = __shfl_xor(best, o2, 64);
        const int oj = __shfl_xor(bj, o2, 64);
        if (ob > best || (ob == best && oj < bj)) {
          best = ob;
          bj = oj;
        }
      }
      if (t == 0) {
        misc[0] = tot;
        misc[2] = (double)bj;
      }
    }
    __syncthreads();
    const double total = misc[0];
    const int piv = (int)misc[2];
    if (total <= prm.tol2) break;
    if (r == kPlrRC) {
      r = kPlrRC + 1;
      break;
    }
    if (t < s) q[t] = R[piv * ld + t];
    __syncthreads();
    if (t < r) {
      double acc = 0.0;
      for (int i = 0; i < s; ++i) acc += Q[t * s + i] * q[i];
      h[t] = acc;
    }
    __syncthreads();
    if (t < s) {
      double v = q[t];
      for (int c = 0; c < r; ++c) v -= h[c] * Q[c * s + t];
      q[t] = v;
    }
    __syncthreads();
    if (t < 64) {
      double acc = 0.0;
      for (int i = t; i < s; i += 64) acc += q[i] * q[i];
      acc = wave_sum(acc);
      if (t == 0) misc[1] = acc;
    }
    __syncthreads();
    const double inv = 1.0 / sqrt(misc[1]);
    if (t < s) {
      const double v = q[t] * inv;
      q[t] = v;
      Q[r * s + t] = v;
    }
    __syncthreads();
    if (t < s) {
      double dot = 0.0;
      for (int i = 0; i < s; ++i) dot += q[i] * R[t * ld + i];
      for (int i = 0; i < s; ++i) R[t * ld + i] -= dot * q[i];
    }
    __syncthreads();
    ++r;
  }
  const int rr = r <= kPlrRC ? r : 0;  // factors kept (none past the cap)
  CT* U = rec + plr_block_off(mp, jb.d, jb.g, jb.side);
  CT* Vt = U + (int64_t)s * kPlrRC;
  for (int e = t; e < s * kPlrRC; e += kPlrThreads) {
    const int i = e / kPlrRC, c = e % kPlrRC;
    const int b = c >> 4, w = c & 15;
    const int rho = 16 * b + (w >> 2) + 4 * (w & 3);  // U'[i][16b + 4a + v] = U[i][16b + a + 4v]
    U[e] = rho < rr ? (CT)Q[rho * s + i] : (CT)0;
  }
  for (int e = t; e < kPlrRC * s; e += kPlrThreads) {
    const int rho = e / s, j = e % s;
    double acc = 0.0;
    if (rho < rr)
      for (int i = 0; i < s; ++i) acc += Q[rho * s + i] * Pk[(int64_t)(row0 + i) * mp + col0 + j];
    Vt[e] = (CT)acc;
  }
  if (t == 0) prm.ranks[prm.rank_off[jb.op] + jb.k * kPlrRankSlots + plr_rank_index(jb.d, jb.g, jb.side)] = r;
}

// Four consecutive state elements of one row through a buffer resource; an
// offset of 2^31 or more lies past the resource (whose size is below 2^31) and
// reads as zero, and a store to it is dropped.
template <typename X>
struct Row4;
template <>
struct Row4<float> {
  using T = f32x4;
  static __device__ __forceinline__ T ld(const __amdgpu_buffer_rsrc_t& rs, uint32_t off) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  }
  static __device__ __forceinline__ void st(const T& v, const __amdgpu_buffer_rsrc_t& rs, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, off, 0, 0);
  }
};
template <>
struct Row4<double> {
  using T = f64x4;
  static __device__ __forceinline__ T ld(const __amdgpu_buffer_rsrc_t& rs, uint32_t off) {
    const u32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    const u32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u, 0, 0);
    typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));
    const u32x8 w{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(T, w);
  }
  static __device__ __forceinline__ void st(const T& v, const __amdgpu_buffer_rsrc_t& rs, uint32_t off) {
    typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));
    const u32x8 w = __builtin_bit_cast(u32x8, v);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[0], w[1], w[2], w[3]}, rs, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[4], w[5], w[6], w[7]}, rs, off + 16u, 0, 0);
  }
};

template <typename X>
__device__ __forceinline__ typename Row4<X>::T ld4(const X* p) {
  return *reinterpret_cast<const typename Row4<X>::T*>(p);
}

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One PLR stage over a unit of 4 NT 16 rows of one sequence (NT = 2 for FP32,
// 1 for FP64): each wave owns NT blocks of 16 consecutive rows and computes
// them alone (no LDS). In the 16 x 16 x 4 products the time rows are the N
// side; K runs over 16 columns of a leaf or of an off-diagonal block (lane
// group a taking columns 4a .. 4a + 3) and over ranks.
//   Z = X_s[:, J] V: the rows of the product are ranks; the A-row to rank map
//       is chosen so that lane group a holds ranks a + 4v, v < 4.
//   y[:, I] = x[:, I] + X_s[:, I] L^T + sum over levels of Z U^T, the Z
//       registers used as B operands as they are; the A-row to output map
//       makes lane group a hold outputs 4a .. 4a + 3.
// Leaves are visited in order. Lower-triangular forms take one sweep (below);
// otherwise the Z of a block is formed when the leaf sweep opens its row range.
template <int MP, typename X>
__global__ __launch_bounds__(kPlrThreads) void k_stage_plr(PlrStageParams prm) {
  using V4 = typename Row4<X>::T;
  using Acc = V4;
  constexpr bool F64 = sizeof(X) == 8;
  constexpr int D = plr_levels(MP), NL = MP / kPlrLeaf;
  constexpr int NT = F64 ? 1 : 2;
  constexpr uint32_t ES = sizeof(X);
  const PlrUnit un = prm.units[blockIdx.x];
  const SeqDev sq = prm.seqs[un.seq];
  const int64_t L = sq.L, sh = (int64_t)1 << prm.k;
  const X* rec = reinterpret_cast<const X*>(prm.rec) + prm.rec_off[sq.op] + (int64_t)prm.k * plr_rec_elems(MP);
  const int32_t* rk = prm.ranks + prm.rank_off[sq.op] + prm.k * kPlrRankSlots;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R = lane & 15, ga = lane >> 4;
  // phase A: A-row R holds rank sigA(R) of its 16; phase B: output sigB(R) of its leaf
  const int sigA = F64 ? R : (R >> 2) + 4 * (R & 3);
  const int sigB = F64 ? 4 * (R & 3) + (R >> 2) : R;

  const uint32_t nrec = (uint32_t)L * (uint32_t)(MP * ES);
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<X*>(reinterpret_cast<const X*>(prm.xin) + sq.x_off), (short)0, (int)nrec, kBufferWord3);
  const auto rout = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<X*>(prm.xout) + sq.x_off, (short)0,
                                                      (int)nrec, kBufferWord3);
  // per time block: byte offsets of row l and of row l - 2^k (bit 31: none)
  uint32_t orow[NT], osh[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int64_t l = (int64_t)un.row0 + (wave * NT + nt) * 16 + R;
    const int64_t ls = l - sh;
    // (exactly 2^31 when out of range: adding a column offset keeps it there)
    orow[nt] = l < L ? (uint32_t)l * (uint32_t)(MP * ES) : 0x80000000u;
    osh[nt] = ls >= 0 && l < L ? (uint32_t)ls * (uint32_t)(MP * ES) : 0x80000000u;
  }
  Acc z[D][NT][2];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) z[d][nt][0] = z[d][nt][1] = Acc{};

  // Lower-triangular forms (every upper block empty, as for all powers of a
  // lower-triangular Abar): one sweep over the leaves reads each 16-column
  // chunk of X_s once. At level d the chunk adds into the Z of the node whose
  // left half holds it; a leaf in a right half uses the Z its node finished
  // over the left half, so one Z per level is live.
  bool lower = true;
#pragma unroll
  for (int d = 1; d <= D; ++d)
    for (int g = 0; g < (1 << (d - 1)); ++g) lower = lower && rk[plr_rank_index(d, g, 1)] == 0;
  if (lower) {
    for (int f = 0; f < NL; ++f) {
      const int i0 = f * kPlrLeaf;
      const uint32_t cb = (uint32_t)(i0 + 4 * ga) * ES;
      Acc y[NT];
      V4 xs[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        y[nt] = Row4<X>::ld(rin, orow[nt] + cb);
        xs[nt] = Row4<X>::ld(rin, osh[nt] + cb);
      }
      const V4 la = ld4(rec + plr_leaf_off(MP) + (int64_t)f * kPlrLeaf * kPlrLeaf + sigB * kPlrLeaf + 4 * ga);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) y[nt] = mfma4(la[v], xs[nt][v], y[nt]);
#pragma unroll
      for (int d = 1; d <= D; ++d) {  // right halves: y += U Z
        const int h = NL >> d, hi = f / h;
        if (!(hi & 1)) continue;
        const int r = rk[plr_rank_index(d, hi >> 1, 0)];
        if (r <= 0 || r > kPlrRC) continue;
        const X* U = rec + plr_block_off(MP, d, hi >> 1, 0) + (int64_t)((f % h) * kPlrLeaf + sigB) * kPlrRC;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (16 * b >= r) break;
          const V4 ua = ld4(U + 16 * b + 4 * ga);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (16 * b + 4 * v >= r) break;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) y[nt] = mfma4(ua[v], z[d - 1][nt][b][v], y[nt]);
          }
        }
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) Row4<X>::st(y[nt], rout, orow[nt] + cb);
#pragma unroll
      for (int d = 1; d <= D; ++d) {  // left halves: Z += X_s[:, chunk] V[chunk, :]
        const int h = NL >> d, hi = f / h;
        if (hi & 1) continue;
        if (f % h == 0) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) z[d - 1][nt][0] = z[d - 1][nt][1] = Acc{};
        }
        const int r = rk[plr_rank_index(d, hi >> 1, 0)];
        if (r <= 0 || r > kPlrRC) continue;
        const int s = MP >> d;
        const X* Vt = rec + plr_block_off(MP, d, hi >> 1, 0) + (int64_t)s * kPlrRC + (f % h) * kPlrLeaf + 4 * ga;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (16 * b >= r) break;
          const V4 va = ld4(Vt + (int64_t)(16 * b + sigA) * s);
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) z[d - 1][nt][b] = mfma4(va[v], xs[nt][v], z[d - 1][nt][b]);
        }
      }
    }
    return;
  }

  for (int f = 0; f < NL; ++f) {
    // phase A: blocks whose row range opens at leaf f
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const int h = NL >> d;  // leaves per half at level d
      if (f % h != 0) continue;
      const int hi = f / h, side = (hi & 1) ? 0 : 1, gg = hi >> 1;
      const int r = rk[plr_rank_index(d, gg, side)];
      const int s = MP >> d;
      const int j0 = (hi ^ 1) * h * kPlrLeaf;
      const X* Vt = rec + plr_block_off(MP, d, gg, side) + (int64_t)s * kPlrRC;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) z[d - 1][nt][0] = z[d - 1][nt][1] = Acc{};
      if (r <= 0 || r > kPlrRC) continue;
      const int nrb = (r + 15) >> 4;
      for (int jc = 0; jc < s; jc += 16) {
        const uint32_t cb = (uint32_t)(j0 + jc + 4 * ga) * ES;
        V4 xs[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) xs[nt] = Row4<X>::ld(rin, osh[nt] + cb);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (b >= nrb) break;
          const V4 va = ld4(Vt + (int64_t)(16 * b + sigA) * s + jc + 4 * ga);
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) z[d - 1][nt][b] = mfma4(va[v], xs[nt][v], z[d - 1][nt][b]);
        }
      }
    }
    // phase B: the 16 outputs of leaf f
    const int i0 = f * kPlrLeaf;
    const uint32_t cb = (uint32_t)(i0 + 4 * ga) * ES;
    Acc y[NT];
    V4 xs[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      y[nt] = Row4<X>::ld(rin, orow[nt] + cb);
      xs[nt] = Row4<X>::ld(rin, osh[nt] + cb);
    }
    const V4 la = ld4(rec + plr_leaf_off(MP) + (int64_t)f * kPlrLeaf * kPlrLeaf + sigB * kPlrLeaf + 4 * ga);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) y[nt] = mfma4(la[v], xs[nt][v], y[nt]);
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      const int h = NL >> d;
      const int hi = f / h, side = (hi & 1) ? 0 : 1, gg = hi >> 1;
      const int r = rk[plr_rank_index(d, gg, side)];
      if (r <= 0 || r > kPlrRC) continue;
      const X* U = rec + plr_block_off(MP, d, gg, side) + (int64_t)((f % h) * kPlrLeaf + sigB) * kPlrRC;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (16 * b >= r) break;
        const V4 ua = ld4(U + 16 * b + 4 * ga);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (16 * b + 4 * v >= r) break;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) y[nt] = mfma4(ua[v], z[d - 1][nt][b][v], y[nt]);
        }
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) Row4<X>::st(y[nt], rout, orow[nt] + cb);
  }
}

template <typename CT>
hipError_t launch_compress_t(const PlrCompressParams& prm, int n_jobs, int max_s, hipStream_t st) {
  const size_t lds = plr_compress_lds(max_s);
  hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_plr_compress<CT>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plr_compress<CT>, dim3(n_jobs), dim3(kPlrThreads), lds, st, prm);
  return hipGetLastError();
}

template <int MP, typename X>
hipError_t launch_stage_plr_t(const PlrStageParams& prm, hipStream_t st) {
  hipLaunchKernelGGL((k_stage_plr<MP, X>), dim3(prm.n_units), dim3(kPlrThreads), 0, st, prm);
  return hipGetLastError();
}

}  // namespace

size_t plr_compress_lds(int max_s) {
  return sizeof(double) * ((size_t)max_s * (max_s + 1) + 2 * (size_t)max_s + kPlrRC + 8);
}

hipError_t launch_plr_compress(int compute, const PlrCompressParams& prm, int n_jobs, int max_s, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  if (max_s > kPlrMaxS) return hipErrorInvalidValue;
  if (compute == DT_F64) return launch_compress_t<double>(prm, n_jobs, max_s, st);
  if (compute == DT_F32) return launch_compress_t<float>(prm, n_jobs, max_s, st);
  return hipErrorInvalidValue;
}

hipError_t launch_stage_plr(int mp, int compute, const PlrStageParams& prm, hipStream_t st) {
  if (prm.n_units <= 0) return hipSuccess;
  if (compute == DT_F32) {
    switch (mp) {
      case 64: return launch_stage_plr_t<64, float>(prm, st);
      case 128: return launch_stage_plr_t<128, float>(prm, st);
      case 256: return launch_stage_plr_t<256, float>(prm, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (compute == DT_F64) {
    switch (mp) {
      case 64: return launch_stage_plr_t<64, double>(prm, st);
      case 128: return launch_stage_plr_t<128, double>(prm, st);
      case 256: return launch_stage_plr_t<256, double>(prm, st);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ssmc
