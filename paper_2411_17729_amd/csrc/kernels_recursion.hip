// The plain recursion of eq. (1.2), x_n = Abar x_{n-1} + Bbar u_n with
// x_{-1} = 0, kept on the GPU as the comparator of the cascade: one
// workgroup per sequence walks its L dependent steps.
//
// 4*MP threads: thread (r, c) holds the quarter c of row r of Abar in
// registers, the current state lives in LDS, and the four partial dot
// products of a row are combined with cross-lane shuffles. Bbar u for a
// chunk of steps is formed in parallel into LDS before the chunk is walked.
// Every state x_n is written out; y = C x + D u is applied afterwards by the
// projection pass of the stage kernel.
#include "ssm_internal.h"

namespace ssmc {

template <typename T>
__device__ __forceinline__ T rload(const void* src, int dtype, int64_t i) {
  if (dtype == DT_F64) return (T)((const double*)src)[i];
  if (dtype == DT_F32) return (T)((const float*)src)[i];
  const uint32_t b = ((const uint16_t*)src)[i];
  return (T)__uint_as_float(b << 16);
}

template <int MP, typename T>
__global__ __launch_bounds__(4 * MP) void k_recursion(const SeqDev* seqs, const OpDev* ops,
                                                      const double* pw, const double* bbar,
                                                      const void* u, int u_dtype, T* xout) {
  constexpr int Q = MP / 4;
  constexpr int CH = 32;  // steps per chunk of Bbar u
  const SeqDev sq = seqs[blockIdx.x];
  const OpDev o = ops[sq.op];
  if (o.mp != MP) return;
  const int tid = threadIdx.x;
  const int r = tid >> 2, c = tid & 3;
  __shared__ T xs[2][MP];
  __shared__ T vs[CH][MP];

  T a[Q];
  const double* P0 = pw + o.pw + (int64_t)r * MP + c * Q;
#pragma unroll
  for (int j = 0; j < Q; ++j) a[j] = (T)P0[j];
  if (c == 0) xs[0][r] = (T)0;
  int cur = 0;
  const int p = sq.p;
  const double* bb = bbar + o.bbar;
  T* xo = xout + sq.x_off;

  for (int64_t l0 = 0; l0 < sq.L; l0 += CH) {
    __syncthreads();
    for (int e = tid; e < CH * MP; e += 4 * MP) {
      const int tt = e / MP, row = e % MP;
      const int64_t l = l0 + tt;
      T v = 0;
      if (l < sq.L)
        for (int j = 0; j < p; ++j) v += (T)bb[row * p + j] * rload<T>(u, u_dtype, sq.u_off + l * p + j);
      vs[tt][row] = v;
    }
    __syncthreads();
    const int nstep = (int)((sq.L - l0) < CH ? (sq.L - l0) : CH);
    for (int tt = 0; tt < nstep; ++tt) {
      const T* xc = xs[cur] + c * Q;
      T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
      for (int j = 0; j < Q; j += 4) {
        s0 += a[j] * xc[j];
        s1 += a[j + 1] * xc[j + 1];
        s2 += a[j + 2] * xc[j + 2];
        s3 += a[j + 3] * xc[j + 3];
      }
      T sum = (s0 + s1) + (s2 + s3);
      sum += __shfl_xor(sum, 1);
      sum += __shfl_xor(sum, 2);
      if (c == 0) {
        const T xn = sum + vs[tt][r];
        xs[cur ^ 1][r] = xn;
        xo[(l0 + tt) * MP + r] = xn;
      }
      cur ^= 1;
      __syncthreads();
    }
  }
}

template <int MP, typename T>
static hipError_t launch_rec(const SeqDev* seqs, int n_seq, const OpDev* ops, const double* pw,
                             const double* bbar, const void* u, int u_dtype, void* xout,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_recursion<MP, T>), dim3(n_seq), dim3(4 * MP), 0, s, seqs, ops, pw, bbar,
                     u, u_dtype, (T*)xout);
  return hipGetLastError();
}

hipError_t launch_recursion(int mp, int ct, const SeqDev* seqs, int n_seq, const OpDev* ops,
                            const double* pw, const double* bbar, const void* u,
                            int u_dtype, void* xout, hipStream_t s) {
  if (n_seq <= 0) return hipSuccess;
  const bool f64 = ct == DT_F64;
  switch (mp) {
    case 32:
      return f64 ? launch_rec<32, double>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s)
                 : launch_rec<32, float>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s);
    case 64:
      return f64 ? launch_rec<64, double>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s)
                 : launch_rec<64, float>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s);
    case 128:
      return f64 ? launch_rec<128, double>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s)
                 : launch_rec<128, float>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s);
    case 256:
      return f64 ? launch_rec<256, double>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s)
                 : launch_rec<256, float>(seqs, n_seq, ops, pw, bbar, u, u_dtype, xout, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace ssmc
