// Reductions of the reverse-mode pass of the fast cascade.
//
// The adjoint of stage k, x_l <- x_l + P_k x_{l-s} (s = 2^k), hands the
// gradient of P_k = Abar^(2^k) as a sum over time of outer products,
//     dL/dP_k = sum_l g_l^(k+1) (x_{l-s}^(k))^T,
// where g^(k+1) is the gradient w.r.t. the stage's output rows and x^(k) its
// input rows. The same form gives dL/dC = sum_l dy_l x_l^T, dL/dD = sum_l dy_l u_l^T
// and dL/dBbar = sum_l g_l^(0) u_l^T. Each workgroup reduces one chunk of rows
// of one sequence on the matrix cores (FP32 MFMA for FP32 state, FP64 MFMA
// for FP64 state) into a partial; the partials are then summed in FP64.
#include <type_traits>

#include "ssm_internal.h"
#include "stage_common.h"

namespace ssmc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename X>
__device__ __forceinline__ X red_load(const void* p, int dtype, int64_t i) {
  if (dtype == DT_F64) return (X)((const double*)p)[i];
  if (dtype == DT_F32) return (X)((const float*)p)[i];
  return (X)__uint_as_float(((uint32_t)((const uint16_t*)p)[i]) << 16);
}

template <typename X>
struct RedMfma;
template <>
struct RedMfma<float> {
  using Acc = f32x4;
  static __device__ __forceinline__ Acc run(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct RedMfma<double> {
  using Acc = f64x4;
  static __device__ __forceinline__ Acc run(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

// One row source: pointer, element type, element offset of the sequence's
// row 0, and row width (= row stride).
template <typename X>
struct RowSrc {
  const void* p;
  int dtype;
  int width;
  int64_t off;
  __device__ __forceinline__ X at(int64_t row, int col) const {
    return red_load<X>(p, dtype, off + row * (int64_t)width + col);
  }
};

template <int MP, typename X>
__device__ __forceinline__ RowSrc<X> row_src(const RedParams& prm, const SeqDev& sq, int kind,
                                             const void* state_base) {
  constexpr int sdt = sizeof(X) == 8 ? DT_F64 : DT_F32;
  RowSrc<X> r;
  if (kind == RS_STATE) {
    r.p = state_base;
    r.dtype = sdt;
    r.width = MP;
    r.off = sq.x_off;
  } else if (kind == RS_U) {
    r.p = prm.u;
    r.dtype = prm.u_dtype;
    r.width = sq.p;
    r.off = sq.u_off;
  } else {
    r.p = prm.dy;
    r.dtype = sdt;
    r.width = sq.q;
    r.off = sq.y_off;
  }
  return r;
}

template <int MP, typename X>
__global__ __launch_bounds__(256) void k_outer(RedParams prm) {
  using M = RedMfma<X>;
  using Acc = typename M::Acc;
  constexpr int TO = sizeof(X) == 8 ? 64 : 128;  // output tile edge
  constexpr int WT = TO / 2;                     // per-wave edge (2 x 2 waves)
  constexpr int NB = WT / 16;                    // 16x16 blocks per wave edge
  constexpr int KT = 16;                         // rows per LDS step
  constexpr int PADK = 4;
  __shared__ X As[KT][TO + PADK];
  __shared__ X Bs[KT][TO + PADK];

  const RedChunk ch = prm.chunks[blockIdx.x];
  const SeqDev sq = prm.seqs[ch.seq];
  const bool first = prm.a_first && prm.k >= 0 && prm.k == sq.last;
  RowSrc<X> A = row_src<MP, X>(prm, sq, prm.a_kind, first ? prm.a_first : prm.a_base);
  RowSrc<X> B = row_src<MP, X>(prm, sq, prm.b_kind, prm.b_base);
  const int wa = A.width, wb = B.width;
  const int ntb = (wb + TO - 1) / TO;
  const int ta = blockIdx.y / ntb, tb = blockIdx.y % ntb;
  const int a0 = ta * TO, b0 = tb * TO;
  if (a0 >= wa) return;
  X* part = reinterpret_cast<X*>(prm.partial) + (int64_t)ch.slot * prm.slot_stride;

  const bool active = !(prm.check_last && prm.k > sq.last);
  const int64_t s = prm.k >= 0 ? ((int64_t)1 << prm.k) : 0;
  int64_t lo = ch.row0;
  if (lo < s) lo = s;
  const int64_t hi = (int64_t)ch.row0 + ch.nrows;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;
  Acc acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = Acc{};

  if (active) {
    for (int64_t l0 = lo; l0 < hi; l0 += KT) {
      __syncthreads();
      for (int e = tid; e < KT * TO; e += 256) {
        const int kk = e / TO, i = e % TO;
        const int64_t l = l0 + kk;
        const bool in = l < hi;
        As[kk][i] = (in && a0 + i < wa) ? A.at(l, a0 + i) : (X)0;
        Bs[kk][i] = (in && b0 + i < wb) ? B.at(l - s, b0 + i) : (X)0;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KT; ks += 4) {
        X af[NB], bf[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) af[i] = As[ks + lg][wr * WT + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < NB; ++j) bf[j] = Bs[ks + lg][wc * WT + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = M::run(af[i], bf[j], acc[i][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int c = b0 + wc * WT + j * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = a0 + wr * WT + i * 16 + M::row(lg, v);
        if (r < wa && c < wb) part[(int64_t)r * wb + c] = acc[i][j][v];
      }
    }
  }
}

template <int MP, typename X>
static hipError_t launch_outer_t(const RedParams& prm, int tiles_y, hipStream_t s) {
  if (prm.n_chunks <= 0 || tiles_y <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_outer<MP, X>), dim3(prm.n_chunks, tiles_y), dim3(256), 0, s, prm);
  return hipGetLastError();
}

// Thin reductions (dC = sum dy x^T, dD = sum dy u^T, dL/dBbar = sum g u^T):
// one side of the outer product is at most 16 wide. Thread t takes column
// t mod W' of the wide side (W' the power of two >= its width) and every
// (256 / W')-th row of the chunk, so a row of the wide side is read with one
// coalesced access per thread. The narrow rows (the same for every thread of
// a row) are staged in LDS 64 rows at a time, each element loaded once by
// the workgroup, and read back as broadcasts. Each thread keeps 16 sums,
// added over the row phases through LDS at the end.
template <int MP, typename X>
__global__ __launch_bounds__(256) void k_outer_thin(RedParams prm) {
  constexpr int NN = 16, G = 64;
  __shared__ X red[NN][256];
  __shared__ X nsm[G][NN];
  const RedChunk ch = prm.chunks[blockIdx.x];
  const SeqDev sq = prm.seqs[ch.seq];
  const bool first = prm.a_first && prm.k >= 0 && prm.k == sq.last;
  const RowSrc<X> A = row_src<MP, X>(prm, sq, prm.a_kind, first ? prm.a_first : prm.a_base);
  const RowSrc<X> B = row_src<MP, X>(prm, sq, prm.b_kind, prm.b_base);
  const bool a_narrow = prm.a_kind != RS_STATE;
  const RowSrc<X>& Nw = a_narrow ? A : B;  // narrow side
  const RowSrc<X>& Ww = a_narrow ? B : A;  // wide side
  const int nw = Nw.width, ww = Ww.width;
  int wp = 1;
  while (wp < ww) wp <<= 1;
  const int phases = 256 / wp;
  const int t = threadIdx.x, c = t % wp, ph = t / wp;
  X acc[NN];
#pragma unroll
  for (int j = 0; j < NN; ++j) acc[j] = (X)0;
  // (uniform over the workgroup: every thread meets the same barriers)
  const bool active = !(prm.check_last && prm.k > sq.last);
  const int64_t s = prm.k >= 0 ? ((int64_t)1 << prm.k) : 0;
  int64_t lo = ch.row0;
  if (lo < s) lo = s;
  const int64_t hi = (int64_t)ch.row0 + ch.nrows;
  if (active) {
    // B rows are shifted by s: the wide side's when A is narrow, else the narrow side's
    const int64_t sw = a_narrow ? s : 0, sn = a_narrow ? 0 : s;
    for (int64_t base = lo; base < hi; base += G) {
      const int nr = (int)(hi - base < G ? hi - base : G);
      for (int e = t; e < nr * nw; e += 256) {
        const int r = e / nw, j = e - r * nw;
        nsm[r][j] = Nw.at(base + r - sn, j);
      }
      __syncthreads();
      if (c < ww) {
        // eight rows of the thread in flight at a time
        int r = ph;
        for (; r + 7 * phases < nr; r += 8 * phases) {
          X wv[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) wv[i] = Ww.at(base + r + i * phases - sw, c);
#pragma unroll
          for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < NN; ++j)
              if (j < nw) acc[j] += nsm[r + i * phases][j] * wv[i];
        }
        for (; r < nr; r += phases) {
          const X wv = Ww.at(base + r - sw, c);
#pragma unroll
          for (int j = 0; j < NN; ++j)
            if (j < nw) acc[j] += nsm[r][j] * wv;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < NN; ++j) red[j][t] = acc[j];
  __syncthreads();
  X* part = reinterpret_cast<X*>(prm.partial) + (int64_t)ch.slot * prm.slot_stride;
  for (int e = t; e < nw * ww; e += 256) {
    const int j = e / ww, cc = e % ww;
    X v = (X)0;
    for (int q = 0; q < phases; ++q) v += red[j][q * wp + cc];
    // output rows follow A: (narrow j, wide cc) when A is narrow, else (cc, j)
    if (a_narrow) part[(int64_t)j * B.width + cc] = v;
    else part[(int64_t)cc * B.width + j] = v;
  }
}

template <int MP, typename X>
static hipError_t launch_outer_thin_t(const RedParams& prm, hipStream_t s) {
  if (prm.n_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_outer_thin<MP, X>), dim3(prm.n_chunks), dim3(256), 0, s, prm);
  return hipGetLastError();
}

hipError_t launch_outer_thin(int mp, int state_f64, const RedParams& prm, hipStream_t s) {
  switch (mp) {
    case 32: return state_f64 ? launch_outer_thin_t<32, double>(prm, s) : launch_outer_thin_t<32, float>(prm, s);
    case 64: return state_f64 ? launch_outer_thin_t<64, double>(prm, s) : launch_outer_thin_t<64, float>(prm, s);
    case 128: return state_f64 ? launch_outer_thin_t<128, double>(prm, s) : launch_outer_thin_t<128, float>(prm, s);
    case 256: return state_f64 ? launch_outer_thin_t<256, double>(prm, s) : launch_outer_thin_t<256, float>(prm, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_outer(int mp, int state_f64, const RedParams& prm, int tiles_y,
                        hipStream_t s) {
  switch (mp) {
    case 32: return state_f64 ? launch_outer_t<32, double>(prm, tiles_y, s)
                              : launch_outer_t<32, float>(prm, tiles_y, s);
    case 64: return state_f64 ? launch_outer_t<64, double>(prm, tiles_y, s)
                              : launch_outer_t<64, float>(prm, tiles_y, s);
    case 128: return state_f64 ? launch_outer_t<128, double>(prm, tiles_y, s)
                               : launch_outer_t<128, float>(prm, tiles_y, s);
    case 256: return state_f64 ? launch_outer_t<256, double>(prm, tiles_y, s)
                               : launch_outer_t<256, float>(prm, tiles_y, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// The state-by-state reduction dL/dP_k (FP32 state): partial[slot] = sum over
// the chunk's rows l of A_l B_{l-s}^T, A and B rows of MP floats. Operands
// come straight from memory: lane (i, kk) of a wave loads V consecutive entries
// of row l + kk (a 16- or 8-byte piece, coalesced across the 16 lanes of a
// row), and entry c of that piece feeds MFMA block c, so block c's output row
// i is state index base + V i + c. Four rows per FP32 16x16x4 MFMA step; four
// waves cover a TO x TO output tile.
// ---------------------------------------------------------------------------
template <int MP>
__global__ __launch_bounds__(256) void k_outer_ss(RedParams prm) {
  constexpr int TO = MP < 128 ? MP : 128;  // output tile edge
  constexpr int WT = TO / 2;               // per-wave edge (2 x 2 waves)
  constexpr int V = WT / 16;               // entries per lane load (2 or 4)
  using VT = typename std::conditional<V == 4, f32x4, float2>::type;
  const RedChunk ch = prm.chunks[blockIdx.x];
  const SeqDev sq = prm.seqs[ch.seq];
  float* part = reinterpret_cast<float*>(prm.partial) + (int64_t)ch.slot * prm.slot_stride;
  constexpr int ntb = MP / TO;
  const int ta = blockIdx.y / ntb, tb = blockIdx.y % ntb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, kk = lane >> 4;
  const int abase = ta * TO + wr * WT, bbase = tb * TO + wc * WT;

  f32x4 acc[V][V];
#pragma unroll
  for (int a = 0; a < V; ++a)
#pragma unroll
    for (int b = 0; b < V; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const bool first = prm.a_first && prm.k >= 0 && prm.k == sq.last;
  const bool active = !(prm.check_last && prm.k > sq.last);
  const int64_t sh = prm.k >= 0 ? ((int64_t)1 << prm.k) : 0;
  int64_t lo = ch.row0;
  if (lo < sh) lo = sh;  // rows without a partner contribute nothing
  const int64_t hi = (int64_t)ch.row0 + ch.nrows;
  if (active && lo < hi) {
    // rows through buffer resources over the sequence's L x MP block (the
    // host keeps L MP 4 < 2^31): rows from hi on get an offset past the end
    // and read as zero, with no branch (a branch would make the compiler wait
    // for each load where it is issued)
    const uint32_t nrec = (uint32_t)sq.L * (uint32_t)(MP * 4);
    const auto rA = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(reinterpret_cast<const float*>(first ? prm.a_first : prm.a_base) + sq.x_off), (short)0,
        (int)nrec, kBufferWord3);
    const auto rB = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(reinterpret_cast<const float*>(prm.b_base) + sq.x_off), (short)0, (int)nrec, kBufferWord3);
    const uint32_t ca = (uint32_t)(abase + V * lr) * 4u, cb = (uint32_t)(bbase + V * lr) * 4u;
    auto ld = [&](const __amdgpu_buffer_rsrc_t& rs, uint32_t col, int64_t row, bool ok) -> VT {
      const uint32_t off = ((uint32_t)row * (uint32_t)(MP * 4) + col) | (ok ? 0u : 0x80000000u);
      if constexpr (V == 4) {
        return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
      } else {
        return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
      }
    };
    // eight rows (two MFMA steps of four) per register set; two sets in
    // turn, each loaded while the other is contracted (unrolled so that no
    // register is copied, which would wait for its load where it is issued)
    VT xa[2][2], xb[2][2];
    auto load8 = [&](int set, int64_t l) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t row = l + 4 * h + kk;
        xa[set][h] = ld(rA, ca, row, row < hi);
        xb[set][h] = ld(rB, cb, row - sh, row < hi);
      }
    };
    auto mfma8 = [&](int set) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int a = 0; a < V; ++a)
#pragma unroll
          for (int b = 0; b < V; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[set][h][a], xb[set][h][b], acc[a][b], 0, 0, 0);
    };
    // the scheduling fences keep each set's loads ahead of the other set's
    // products (left alone, the compiler sinks them next to their use)
    load8(0, lo);
    for (int64_t l = lo; l < hi; l += 16) {
      load8(1, l + 8);
      __builtin_amdgcn_sched_barrier(0);
      mfma8(0);
      __builtin_amdgcn_sched_barrier(0);
      load8(0, l + 16);
      __builtin_amdgcn_sched_barrier(0);
      mfma8(1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // accumulator entry v of block (a, b): output row 4 kk + v, column lr
#pragma unroll
  for (int a = 0; a < V; ++a)
#pragma unroll
    for (int b = 0; b < V; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = abase + V * (4 * kk + v) + a, c = bbase + V * lr + b;
        part[(int64_t)r * MP + c] = acc[a][b][v];
      }
}

hipError_t launch_outer_ss(int mp, const RedParams& prm, hipStream_t s) {
  if (prm.n_chunks <= 0) return hipSuccess;
  switch (mp) {
    case 64: hipLaunchKernelGGL(k_outer_ss<64>, dim3(prm.n_chunks, 1), dim3(256), 0, s, prm); break;
    case 128: hipLaunchKernelGGL(k_outer_ss<128>, dim3(prm.n_chunks, 1), dim3(256), 0, s, prm); break;
    case 256: hipLaunchKernelGGL(k_outer_ss<256>, dim3(prm.n_chunks, 4), dim3(256), 0, s, prm); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The same reduction for plans whose stage contractions run in BF16: the
// products of dL/dP_k on the BF16 matrix cores, from the FP32 state rounded
// to BF16 (the operand type of the stages themselves), accumulated in FP32
// within a chunk and in FP64 across chunks. One workgroup of eight waves
// takes one chunk and the whole MP x MP output, so every state row is read
// once; waves split it 2 (rows) x 4 (columns). The time rows are the MFMA
// contraction (32 per step); a step's 32 rows of both operands are loaded
// (a step ahead), rounded and written to LDS transposed, entry-major, so a
// lane's operand (8 consecutive time rows of one entry) is 16 contiguous
// bytes. Thread t loads rows 2 (t % 16) and 2 (t % 16) + 1 of entries
// MP / 32 (t / 16) .. + MP / 32 - 1 and writes each entry's row pair as one
// 32-bit word; the entry order is rotated by half a group for odd groups so
// that the two half-waves of a write fall in different banks.
// ---------------------------------------------------------------------------
template <int MP>
__global__ __launch_bounds__(512, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_outer_bf16(RedParams prm) {
  static_assert(MP == 128 || MP == 256, "16-byte loads of MP / 32 entries per thread");
  constexpr int KR = 32;                 // time rows per step
  constexpr int RS = KR + 8;             // LDS row stride (BF16 entries; 80 bytes)
  constexpr int EG = MP / 32;            // entries of a thread's load group
  constexpr int BA = MP / 32, BB = MP / 64;  // MFMA blocks of a wave (rows, columns)
  constexpr int OPS = MP * RS;           // one operand buffer (BF16 entries)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_obf[];
  __bf16* lds = reinterpret_cast<__bf16*>(smem_obf);  // [2 steps][A, B][MP][RS]

  const RedChunk ch = prm.chunks[blockIdx.x];
  const SeqDev sq = prm.seqs[ch.seq];
  float* part = reinterpret_cast<float*>(prm.partial) + (int64_t)ch.slot * prm.slot_stride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int aw0 = (wave >> 2) * (MP / 2), bw0 = (wave & 3) * (MP / 4);

  f32x4 acc[BA][BB];
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const bool first = prm.a_first && prm.k >= 0 && prm.k == sq.last;
  const bool active = !(prm.check_last && prm.k > sq.last);
  const int64_t sh = prm.k >= 0 ? ((int64_t)1 << prm.k) : 0;
  int64_t lo = ch.row0;
  if (lo < sh) lo = sh;  // rows without a partner contribute nothing
  const int64_t hi = (int64_t)ch.row0 + ch.nrows;
  if (active && lo < hi) {
    // rows through buffer resources over the sequence's L x MP block (the
    // host keeps L MP 4 < 2^31): rows from hi on get an offset past the end
    // and read as zero, with no branch (a branch would make the compiler
    // wait for each step's loads where they are issued)
    const uint32_t nrec = (uint32_t)sq.L * (uint32_t)(MP * 4);
    const auto ra_ = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(reinterpret_cast<const float*>(first ? prm.a_first : prm.a_base) + sq.x_off), (short)0,
        (int)nrec, kBufferWord3);
    const auto rb_ = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(reinterpret_cast<const float*>(prm.b_base) + sq.x_off), (short)0, (int)nrec, kBufferWord3);
    const int rp = threadIdx.x & 15, eg = threadIdx.x >> 4;
    const int e0 = eg * EG;
    constexpr int NV = EG / 4;  // 16-byte loads per row of a thread's group
    f32x4 ra[2][NV], rb[2][NV];
    auto load = [&](int64_t l0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t l = l0 + 2 * rp + h;
        const uint32_t oob = l < hi ? 0u : 0x80000000u;
        const uint32_t oa = ((uint32_t)l * (uint32_t)MP + (uint32_t)e0) * 4u | oob;
        const uint32_t ob = ((uint32_t)(l - sh) * (uint32_t)MP + (uint32_t)e0) * 4u | oob;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          ra[h][v] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra_, oa + 16 * v, 0, 0));
          rb[h][v] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb_, ob + 16 * v, 0, 0));
        }
      }
    };
    auto stage = [&](int buf) {
      __bf16* la = lds + (size_t)buf * 2 * OPS;
      __bf16* lb = la + OPS;
#pragma unroll
      for (int i = 0; i < EG; ++i) {
        const int ei = (i + (eg & 1) * (EG / 2)) % EG;  // rotated entry order
        const int e = e0 + ei;
        const float a0 = ra[0][ei / 4][ei % 4], a1 = ra[1][ei / 4][ei % 4];
        const float b0 = rb[0][ei / 4][ei % 4], b1 = rb[1][ei / 4][ei % 4];
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        const bf16x2 pa{(__bf16)a0, (__bf16)a1}, pb{(__bf16)b0, (__bf16)b1};  // round to nearest even
        *reinterpret_cast<bf16x2*>(la + e * RS + 2 * rp) = pa;
        *reinterpret_cast<bf16x2*>(lb + e * RS + 2 * rp) = pb;
      }
    };
    int64_t l0 = lo;
    load(l0);
    int buf = 0;
    for (; l0 < hi; l0 += KR) {
      stage(buf);
      if (l0 + KR < hi) load(l0 + KR);  // (uniform) the next step, in flight during this one
      __syncthreads();
      const __bf16* la = lds + (size_t)buf * 2 * OPS;
      const __bf16* lb = la + OPS;
      bf16x8 bo[BB];
#pragma unroll
      for (int b = 0; b < BB; ++b) bo[b] = *reinterpret_cast<const bf16x8*>(lb + (bw0 + 16 * b + r) * RS + 8 * g);
#pragma unroll
      for (int a = 0; a < BA; ++a) {
        const bf16x8 ao = *reinterpret_cast<const bf16x8*>(la + (aw0 + 16 * a + r) * RS + 8 * g);
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao, bo[b], acc[a][b], 0, 0, 0);
      }
      buf ^= 1;
    }
  }
  // accumulator entry v of block (a, b): output row 4 g + v, column r
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ro = aw0 + 16 * a + 4 * g + v, co = bw0 + 16 * b + r;
        part[(int64_t)ro * MP + co] = acc[a][b][v];
      }
}

size_t outer_bf16_lds(int mp) { return (size_t)2 * 2 * mp * (32 + 8) * sizeof(__bf16); }

hipError_t launch_outer_bf16(int mp, const RedParams& prm, hipStream_t s) {
  if (prm.n_chunks <= 0) return hipSuccess;
  const size_t lds = outer_bf16_lds(mp);
  switch (mp) {
    case 128: {
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_outer_bf16<128>), lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_outer_bf16<128>, dim3(prm.n_chunks), dim3(512), lds, s, prm);
      break;
    }
    case 256: {
      hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_outer_bf16<256>), lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_outer_bf16<256>, dim3(prm.n_chunks), dim3(512), lds, s, prm);
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 sum of the partials of each job (blockIdx.y = job); the summation
// order is fixed, so the result is deterministic.
// ---------------------------------------------------------------------------
template <typename X>
__global__ __launch_bounds__(256) void k_sum(const SumJob* jobs, int k, const X* partial, double* out) {
  // 64 elements per block, the slots split in four interleaved groups whose
  // FP64 sums are added in a fixed order
  __shared__ double red[4][64];
  const SumJob jb = jobs[blockIdx.y];
  if (k > jb.kmax) return;
  const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
  for (int e0 = blockIdx.x * 64; e0 < jb.elems; e0 += gridDim.x * 64) {
    const int e = e0 + el;
    double acc0 = 0.0, acc1 = 0.0;
    if (e < jb.elems) {
      const X* p = partial + jb.slot0 * jb.slot_stride + e;
      int c = grp;
      for (; c + 4 < jb.nslots; c += 8) {
        acc0 += (double)p[(int64_t)c * jb.slot_stride];
        acc1 += (double)p[(int64_t)(c + 4) * jb.slot_stride];
      }
      if (c < jb.nslots) acc0 += (double)p[(int64_t)c * jb.slot_stride];
    }
    red[grp][el] = acc0 + acc1;
    __syncthreads();
    if (grp == 0 && e < jb.elems)
      out[jb.out + (int64_t)k * jb.kstride + e] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
    __syncthreads();
  }
}

hipError_t launch_sum(const SumJob* jobs, int n_jobs, int max_elems, int k, const void* partial,
                      int state_f64, double* out, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  int bx = (max_elems + 63) / 64;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  if (state_f64)
    hipLaunchKernelGGL(k_sum<double>, dim3(bx, n_jobs), dim3(256), 0, s, jobs, k,
                       (const double*)partial, out);
  else
    hipLaunchKernelGGL(k_sum<float>, dim3(bx, n_jobs), dim3(256), 0, s, jobs, k,
                       (const float*)partial, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per parameter set (blockIdx.y): dA = sum over its operators of dA_op,
// dB likewise, dC and dD from the set's own sums; padding cropped; written as
// [dA (m x m) | dB (m x p) | dC (q x m) | dD (q x p)] at the set's offset.
// ---------------------------------------------------------------------------
__global__ void k_scatter(const ScatterJob* jobs, const int32_t* set_ops, const OpDev* ops,
                          const double* g, double* out) {
  const ScatterJob jb = jobs[blockIdx.y];
  const int m = jb.m, mp = jb.mp, p = jb.p, q = jb.q;
  double* dst = out + jb.out;
  const int nA = m * m, nB = m * p, nC = q * m, nD = q * p;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nA + nB + nC + nD;
       e += gridDim.x * blockDim.x) {
    double v = 0.0;
    if (e < nA) {
      const int r = e / m, c = e % m;
      for (int i = 0; i < jb.n_ops; ++i) v += g[ops[set_ops[jb.op_first + i]].g_da + r * mp + c];
    } else if (e < nA + nB) {
      const int f = e - nA, r = f / p, c = f % p;
      for (int i = 0; i < jb.n_ops; ++i) v += g[ops[set_ops[jb.op_first + i]].g_db + r * p + c];
    } else if (e < nA + nB + nC) {
      const int f = e - nA - nB, r = f / m, c = f % m;
      v = jb.dC >= 0 ? g[jb.dC + r * mp + c] : 0.0;
    } else {
      const int f = e - nA - nB - nC;
      v = jb.dD >= 0 ? g[jb.dD + f] : 0.0;
    }
    dst[e] = v;
  }
}

hipError_t launch_scatter(const ScatterJob* jobs, int n_jobs, const int32_t* set_ops,
                          const OpDev* ops, const double* gws, double* out, int max_mp,
                          hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  int bx = (max_mp * max_mp + 255) / 256;
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(k_scatter, dim3(bx, n_jobs), dim3(256), 0, s, jobs, set_ops, ops, gws, out);
  return hipGetLastError();
}

}  // namespace ssmc
