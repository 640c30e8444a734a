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
#include "ssm_internal.h"

namespace ssmc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

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
// FP64 sum of the partials of each job (blockIdx.y = job); the summation
// order is fixed, so the result is deterministic.
// ---------------------------------------------------------------------------
template <typename X>
__global__ void k_sum(const SumJob* jobs, int k, const X* partial, double* out) {
  const SumJob jb = jobs[blockIdx.y];
  if (k > jb.kmax) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < jb.elems; e += gridDim.x * blockDim.x) {
    double acc = 0.0;
    const X* p = partial + jb.slot0 * jb.slot_stride + e;
    for (int c = 0; c < jb.nslots; ++c) acc += (double)p[(int64_t)c * jb.slot_stride];
    out[jb.out + (int64_t)k * jb.kstride + e] = acc;
  }
}

hipError_t launch_sum(const SumJob* jobs, int n_jobs, int max_elems, int k, const void* partial,
                      int state_f64, double* out, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  int bx = (max_elems + 255) / 256;
  if (bx > 256) bx = 256;
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
