// The plain recursion of eq. (1.2), x_n = Abar x_{n-1} + Bbar u_n with
// x_{-1} = 0, kept on the GPU as the comparator of the cascade: one
// workgroup per sequence walks its L dependent steps. Every state x_n is
// written out; y = C x + D u is applied afterwards by the projection pass of
// the stage kernel.
#include "ssm_internal.h"

namespace ssmc {

template <typename T>
__device__ __forceinline__ T rload(const void* src, int dtype, int64_t i) {
  if (dtype == DT_F64) return (T)((const double*)src)[i];
  if (dtype == DT_F32) return (T)((const float*)src)[i];
  const uint32_t b = ((const uint16_t*)src)[i];
  return (T)__uint_as_float(b << 16);
}

// DPP lane moves within a row of 16 lanes: lane i takes the value of lane
// 7 - (i mod 8) of its half row, of i ^ 1, of i ^ 2 (quad permutations)
constexpr int kDppHalfMirror = 0x141, kDppXor1 = 0xB1, kDppXor2 = 0x4E;

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// FP32: 2*MP threads. The eight lanes 8g .. 8g + 7 own rows 4g .. 4g + 3 of
// Abar; lane c of the eight holds, for those rows, the 16-byte column chunks
// c, c + 8, c + 16, ... in registers (MP/2 floats), so at every step one
// 16-byte LDS read of the previous state serves four rows, and the eight
// lanes of a read instruction fetch eight consecutive chunks (no bank
// conflicts). The eight partial sums of a row are combined by a
// reduce-scatter over lanes with three DPP moves, after which lanes c and
// c + 1 (c = 0, 4) of the group hold rows 4g + c/2 and 4g + c/2 + 1, add
// v_n = (Bbar u)_n and write x_n to LDS and to memory. The state is double-buffered in LDS, so a
// step needs one barrier. Bbar u is formed for a chunk of steps at a time
// from u staged in LDS; the next chunk's u is loaded into registers while the
// current chunk is walked.
template <int MP>
__global__ __launch_bounds__(2 * MP) void k_recursion_f32(const SeqDev* seqs, const OpDev* ops,
                                                          const double* pw, const double* bbar,
                                                          const void* u, int u_dtype, float* xout) {
  constexpr int NT = 2 * MP;
  constexpr int NCH = MP / 32;  // 16-byte chunks of columns per lane
  constexpr int CHMAX = 64;     // steps per chunk of Bbar u
  constexpr int PF = 8;         // prefetched u elements per thread
  const SeqDev sq = seqs[blockIdx.x];
  const OpDev o = ops[sq.op];
  if (o.mp != MP) return;
  const int tid = threadIdx.x;
  const int c = tid & 7;
  const int row0 = (tid >> 3) * 4;
  __shared__ __align__(16) float xs[2][MP];
  __shared__ float vs[CHMAX][MP];
  __shared__ float us[PF * NT];

  // Abar in FP32 registers, converted through LDS a quarter of the rows at a
  // time (vs holds CHMAX * MP >= MP * MP / 4 floats)
  float a[4][NCH][4];
  {
    static_assert(CHMAX * MP >= MP * MP / 4, "vs holds a quarter of Abar");
    const double* P0 = pw + o.pw;
    float* stage = &vs[0][0];
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      __syncthreads();
      for (int e = tid; e < MP * MP / 4; e += NT) stage[e] = (float)P0[(int64_t)qd * (MP * MP / 4) + e];
      __syncthreads();
      if (row0 / (MP / 4) == qd) {
        const int lr = row0 - qd * (MP / 4);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < NCH; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) a[r][j][e] = stage[(lr + r) * MP + (c + 8 * j) * 4 + e];
      }
    }
    __syncthreads();
  }
  if (tid < MP) xs[0][tid] = 0.f;
  const int p = sq.p;
  const int64_t L = sq.L;
  const int CH = (PF * NT) / p < CHMAX ? (PF * NT) / p : CHMAX;
  const double* bb = bbar + o.bbar;
  float* xo = xout + sq.x_off;
  const bool hi = (c & 4) != 0, b0 = (c & 1) != 0;
  const int myrow = row0 + (hi ? 2 : 0) + (b0 ? 1 : 0);
  const bool writer = (c & 2) == 0;

  float pf[PF];
  auto prefetch = [&](int64_t l0) {
    const int64_t rows = (L - l0) < CH ? (L - l0) : CH;
    const int n = (int)rows * p;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * NT;
      pf[i] = e < n ? rload<float>(u, u_dtype, sq.u_off + l0 * p + e) : 0.f;
    }
  };
  // Bbar u of the next nrows steps into vs (after the last step's barrier)
  auto stage_v = [&](int nrows) {
    const int n = nrows * p;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * NT;
      if (e < n) us[e] = pf[i];
    }
    __syncthreads();
    for (int e = tid; e < nrows * MP; e += NT) {
      const int tt = e / MP, row = e % MP;
      float v = 0.f;
      for (int j = 0; j < p; ++j) v += (float)bb[row * p + j] * us[tt * p + j];
      vs[tt][row] = v;
    }
    __syncthreads();
  };

  prefetch(0);
  stage_v((int)(L < CH ? L : CH));
  int cur = 0;
  for (int64_t l0 = 0; l0 < L; l0 += CH) {
    const int nstep = (int)((L - l0) < CH ? (L - l0) : CH);
    const bool more = l0 + CH < L;
    if (more) prefetch(l0 + CH);
    for (int tt = 0; tt < nstep; ++tt) {
      // every LDS read of the step (the previous state's chunks and v_n) is
      // issued before the first contraction
      const float4* xc = reinterpret_cast<const float4*>(xs[cur]);
      float4 xv[NCH];
#pragma unroll
      for (int j = 0; j < NCH; ++j) xv[j] = xc[c + 8 * j];
      const float vn = vs[tt][myrow];
      float acc[4][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
#pragma unroll
      for (int j = 0; j < NCH; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc[r][j & 1] += a[r][j][0] * xv[j].x;
          acc[r][j & 1] += a[r][j][1] * xv[j].y;
          acc[r][j & 1] += a[r][j][2] * xv[j].z;
          acc[r][j & 1] += a[r][j][3] * xv[j].w;
        }
      }
      asm volatile("" ::"v"(vn));  // v_n is read by every lane, ahead of the reduction
      const float r0 = acc[0][0] + acc[0][1], r1 = acc[1][0] + acc[1][1];
      const float r2 = acc[2][0] + acc[2][1], r3 = acc[3][0] + acc[3][1];
      // reduce-scatter over the eight lanes of the row group with DPP moves:
      // partner 7 - c (lanes 0-3 keep rows 0, 1; lanes 4-7 rows 2, 3), then
      // c ^ 1 (keep the row of bit 0), then c ^ 2 (the same row)
      float k0 = hi ? r2 : r0, k1 = hi ? r3 : r1;
      const float s0 = hi ? r0 : r2, s1 = hi ? r1 : r3;
      k0 += dpp_f32<kDppHalfMirror>(s0);
      k1 += dpp_f32<kDppHalfMirror>(s1);
      float k = b0 ? k1 : k0;
      const float s = b0 ? k0 : k1;
      k += dpp_f32<kDppXor1>(s);
      k += dpp_f32<kDppXor2>(k);
      if (writer) {
        const float xn = k + vn;
        xs[cur ^ 1][myrow] = xn;
        xo[(l0 + tt) * MP + myrow] = xn;
      }
      cur ^= 1;
      __syncthreads();
    }
    if (more) stage_v((int)((L - l0 - CH) < CH ? (L - l0 - CH) : CH));
  }
}

// FP64 (the F64 plan's comparator): 4*MP threads; thread (r, c) holds the
// quarter c of row r of Abar in registers, the current state lives in LDS,
// and the four partial dot products of a row are combined with cross-lane
// shuffles. Bbar u for a chunk of steps is formed in parallel into LDS before
// the chunk is walked.
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
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((k_recursion_f32<MP>), dim3(n_seq), dim3(2 * MP), 0, s, seqs, ops, pw, bbar, u,
                       u_dtype, (float*)xout);
  else
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
