// FP64 precomputation on the GPU: trapezoidal discretization (§1, the
// formulas after eq. (1.2)), the powers Abar^(2^k) by repeated squaring
// (end of §2, start of §3), and their cast to the stage compute type.
#include <float.h>

#include "ssm_internal.h"

namespace ssmc {

// ---------------------------------------------------------------------------
// Setup of the trapezoid system per operator (blockIdx.y = operator).
//   aug  = [ I - h A | I ]   (mp x 2mp; the padded block of I - hA is I)
//   nmat = I + h A            (mp x mp; zero in the padding)
//   bsc  = delta B            (mp x p)
// For given discrete parameters, Abar goes straight to the k = 0 power slot
// and Bbar to bbar.
// ---------------------------------------------------------------------------
__global__ void k_disc_setup(const OpDev* ops, const OpSrc* src, int given, double* aug,
                             double* nmat, double* bsc, double* pw, double* bbar) {
  const OpDev o = ops[blockIdx.y];
  const OpSrc sp = src[blockIdx.y];
  const int mp = o.mp, m = o.m, p = o.p;
  const double h = 0.5 * o.delta;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = e0; e < (int64_t)mp * mp; e += stride) {
    const int r = (int)(e / mp), c = (int)(e % mp);
    const bool in = r < m && c < m;
    const double a = in ? sp.A[(int64_t)r * m + c] : 0.0;
    const double id = r == c ? 1.0 : 0.0;
    if (given) {
      pw[o.pw + e] = a;
    } else {
      double* ag = aug + o.sc_aug + (int64_t)r * 2 * mp;
      ag[c] = in ? id - h * a : id;
      ag[mp + c] = id;
      nmat[o.sc_n + e] = in ? id + h * a : 0.0;
    }
  }
  for (int64_t e = e0; e < (int64_t)mp * p; e += stride) {
    const int r = (int)(e / p), c = (int)(e % p);
    const double bv = r < m ? sp.B[(int64_t)r * p + c] : 0.0;
    if (given)
      bbar[o.bbar + e] = bv;
    else
      bsc[o.sc_b + e] = o.delta * bv;
  }
}

// Exponential discretization (§5): the augmented matrix E = delta [[A, B], [0,
// 0]] ((m + p) x (m + p), row-major, at zx of the scratch), the larger of its
// 1- and infinity-norms (largest column and row sums of |E|; the adjoint uses
// E^T) for the choice of the scaling, and zeros in the
// padded slots of Abar (P_0) and Bbar that the exponential fills. Workgroup
// (x, op); workgroup (0, 0) also writes the identity of size nid used by the
// Taylor steps.
__global__ void k_zoh_setup(const OpDev* ops, const OpSrc* src, double* zs, double* zid, int nid,
                            double* norms, double* pw, double* bbar) {
  const OpDev o = ops[blockIdx.y];
  const OpSrc sp = src[blockIdx.y];
  const int m = o.m, p = o.p, n = o.zn, mp = o.mp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double* X = zs + o.zx;
  for (int64_t e = e0; e < (int64_t)n * n; e += stride) {
    const int r = (int)(e / n), c = (int)(e % n);
    const double v = r >= m ? 0.0 : c < m ? sp.A[(int64_t)r * m + c] : sp.B[(int64_t)r * p + (c - m)];
    X[e] = o.delta * v;
  }
  for (int64_t e = e0; e < (int64_t)mp * mp; e += stride) pw[o.pw + e] = 0.0;
  for (int64_t e = e0; e < (int64_t)mp * p; e += stride) bbar[o.bbar + e] = 0.0;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int64_t e = threadIdx.x; e < (int64_t)nid * nid; e += blockDim.x)
      zid[e] = (e / nid) == (e % nid) ? 1.0 : 0.0;
  if (blockIdx.x == 0) {
    // column and row sums from the sources (not from X, which other
    // workgroups write)
    double best = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      double sum = 0.0;
      for (int r = 0; r < m; ++r) sum += fabs(c < m ? sp.A[(int64_t)r * m + c] : sp.B[(int64_t)r * p + (c - m)]);
      sum *= fabs(o.delta);
      best = (sum > best || sum != sum) ? sum : best;  // a NaN wins
    }
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
      double sum = 0.0;
      for (int c = 0; c < m; ++c) sum += fabs(sp.A[(int64_t)r * m + c]);
      for (int c = 0; c < p; ++c) sum += fabs(sp.B[(int64_t)r * p + c]);
      sum *= fabs(o.delta);
      best = (sum > best || sum != sum) ? sum : best;
    }
    __shared__ double red[256];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) {
        const double v = red[threadIdx.x + h];
        if (v > red[threadIdx.x] || v != v) red[threadIdx.x] = v;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) norms[blockIdx.y] = red[0];
  }
}

hipError_t launch_zoh_setup(const OpDev* ops, int n_ops, const OpSrc* src, double* zs, double* zid, int nid,
                            double* norms, double* pw, double* bbar, int max_n, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  const int blocks = (max_n * max_n + 255) / 256;
  hipLaunchKernelGGL(k_zoh_setup, dim3(blocks < 256 ? blocks : 256, n_ops), dim3(256), 0, s, ops, src, zs, zid,
                     nid, norms, pw, bbar);
  return hipGetLastError();
}

hipError_t launch_disc_setup(const OpDev* ops, int n_ops, const OpSrc* src, int given,
                             double* aug, double* nmat, double* bsc, double* pw,
                             double* bbar, int max_mp, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  const int blocks = (max_mp * max_mp + 255) / 256;
  hipLaunchKernelGGL(k_disc_setup, dim3(blocks < 256 ? blocks : 256, n_ops), dim3(256), 0, s,
                     ops, src, given, aug, nmat, bsc, pw, bbar);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gauss-Jordan elimination with partial pivoting, one workgroup per operator:
// [M | I] -> [I | M^{-1}], then M^{-1} is copied to its slot. A pivot below
// mp * eps * max|M| marks the operator as numerically singular.
// ---------------------------------------------------------------------------
constexpr int GJ_THREADS = 1024;

__device__ void block_argmax(double v, int idx, double* sv, int* si, double* out_v, int* out_i) {
  // larger value wins; on ties the smaller index
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sv[w] = v;
    si[w] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sv[0];
    int bi = si[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      if (sv[i] > bv || (sv[i] == bv && si[i] < bi)) {
        bv = sv[i];
        bi = si[i];
      }
    }
    *out_v = bv;
    *out_i = bi;
  }
  __syncthreads();
}

__global__ __launch_bounds__(GJ_THREADS) void k_gauss_jordan(const OpDev* ops, double* aug,
                                                             double* minv, int* status, const int32_t* tri) {
  if (tri[blockIdx.x]) return;  // inverted by the triangular path
  const OpDev o = ops[blockIdx.x];
  const int mp = o.mp, W = 2 * mp;
  double* a = aug + o.sc_aug;
  __shared__ double fac[256];
  __shared__ double red_v[GJ_THREADS / 64];
  __shared__ int red_i[GJ_THREADS / 64];
  __shared__ double s_v;
  __shared__ int s_i;
  const int tid = threadIdx.x;

  // scale for the singularity threshold
  double mx = 0.0;
  for (int e = tid; e < mp * mp; e += GJ_THREADS) mx = fmax(mx, fabs(a[(e / mp) * W + (e % mp)]));
  block_argmax(mx, 0, red_v, red_i, &s_v, &s_i);
  const double thresh = (double)mp * DBL_EPSILON * s_v;

  for (int c = 0; c < mp; ++c) {
    double best = -1.0;
    int bi = c;
    for (int r = c + tid; r < mp; r += GJ_THREADS) {
      const double v = fabs(a[(int64_t)r * W + c]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
    block_argmax(best, bi, red_v, red_i, &s_v, &s_i);
    const int piv = s_i;
    if (tid == 0 && !(s_v > thresh)) atomicOr(status, 1);
    if (piv != c) {
      for (int j = tid; j < W; j += GJ_THREADS) {
        const double t0 = a[(int64_t)c * W + j];
        a[(int64_t)c * W + j] = a[(int64_t)piv * W + j];
        a[(int64_t)piv * W + j] = t0;
      }
    }
    __syncthreads();
    const double inv = 1.0 / a[(int64_t)c * W + c];
    __syncthreads();
    for (int j = c + tid; j < W; j += GJ_THREADS) a[(int64_t)c * W + j] *= inv;
    for (int r = tid; r < mp; r += GJ_THREADS) fac[r] = r == c ? 0.0 : a[(int64_t)r * W + c];
    __syncthreads();
    const int span = W - c;
    for (int e = tid; e < mp * span; e += GJ_THREADS) {
      const int r = e / span, j = c + e % span;
      const double f = fac[r];
      if (f != 0.0) a[(int64_t)r * W + j] -= f * a[(int64_t)c * W + j];
    }
    __syncthreads();
  }
  for (int e = tid; e < mp * mp; e += GJ_THREADS)
    minv[o.minv + e] = a[(int64_t)(e / mp) * W + mp + (e % mp)];
}

// Frobenius norms of the powers Abar^(2^k), k = 0..N of every operator (for
// the automatic choice of N), into norms at (sum of N + 1 over the operators
// before) + k. Workgroup (k, op); the sum of squares is reduced in a fixed
// order.
__global__ __launch_bounds__(256) void k_power_norms(const OpDev* ops, const double* pw, double* norms) {
  const int k = blockIdx.x, op = blockIdx.y;
  const OpDev o = ops[op];
  if (k > o.N) return;
  int64_t base = 0;
  for (int i = 0; i < op; ++i) base += ops[i].N + 1;
  const int64_t mm = (int64_t)o.mp * o.mp;
  const double* Pk = pw + o.pw + k * mm;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < mm; e += 256) acc = fma(Pk[e], Pk[e], acc);
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[base + k] = sqrt(red[0]);
}

hipError_t launch_power_norms(const OpDev* ops, int n_ops, int max_N, const double* pw, double* norms,
                              hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_power_norms, dim3(max_N + 1, n_ops), dim3(256), 0, s, ops, pw, norms);
  return hipGetLastError();
}

hipError_t launch_gauss_jordan(const OpDev* ops, int n_ops, double* aug, double* minv,
                               int* status, const int32_t* tri, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gauss_jordan, dim3(n_ops), dim3(GJ_THREADS), 0, s, ops, aug, minv,
                     status, tri);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lower-triangular M = I - h A. Its inverse is lower triangular, found block
// by block: the 32 x 32 diagonal blocks by forward substitution, then by
// doubling the block size, [[X, 0], [Y, Z]]^{-1} = [[X^-1, 0], [-Z^-1 Y X^-1,
// Z^-1]], two FP64 GEMMs per level (jobs gated on tri).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_tri_check(const OpDev* ops, const OpSrc* src, int32_t* tri,
                                                    double* scale) {
  const OpDev o = ops[blockIdx.x];
  const OpSrc sp = src[blockIdx.x];
  const int m = o.m;
  const double h = 0.5 * o.delta;
  // thread (ty, tx): column tx of rows ty, ty + 4, ... (one coalesced row per step)
  const int tx = threadIdx.x & 255, ty = threadIdx.x >> 8;
  int upper = 0;
  double mx = 0.0;
  if (tx < m)
    for (int r = ty; r < m; r += 4) {
      const double a = sp.A[(int64_t)r * m + tx];
      if (tx > r && a != 0.0) upper = 1;
      mx = fmax(mx, fabs((r == tx ? 1.0 : 0.0) - h * a));
    }
  __shared__ int su[1024];
  __shared__ double sm[1024];
  su[threadIdx.x] = upper;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      su[threadIdx.x] |= su[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tri[blockIdx.x] = su[0] ? 0 : 1;
    scale[blockIdx.x] = fmax(sm[0], 1.0);  // the padding adds ones to the diagonal
  }
}

// ops[i].lower = 1 when the FP64 Abar of operator i (its power k = 0) has no
// nonzero entry above the diagonal; then every power Abar^(2^k) is lower
// triangular too.
__global__ __launch_bounds__(1024) void k_mark_lower(OpDev* ops, const double* pw) {
  const OpDev o = ops[blockIdx.x];
  const double* A = pw + o.pw;
  const int mp = o.mp, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave w reads rows w, w + 16, ... whole (coalesced, no data-dependent
  // branch, so the loads of several rows are in flight together)
  int upper = 0;
#pragma unroll 4
  for (int r = wave; r < mp; r += 16) {
    const double* row = A + (int64_t)r * mp;
    for (int c = lane; c < mp; c += 64) upper |= (c > r) & (row[c] != 0.0);
  }
  upper = __syncthreads_or(upper);
  if (threadIdx.x == 0) ops[blockIdx.x].lower = upper ? 0 : 1;
}

hipError_t launch_mark_lower(OpDev* ops, int n_ops, const double* pw, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_lower, dim3(n_ops), dim3(1024), 0, s, ops, pw);
  return hipGetLastError();
}

hipError_t launch_tri_check(const OpDev* ops, int n_ops, const OpSrc* src, int32_t* tri, double* scale,
                            hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_check, dim3(n_ops), dim3(1024), 0, s, ops, src, tri, scale);
  return hipGetLastError();
}

// Workgroup (block row b, operator): thread j < 32 walks column j of the
// block's inverse in registers, x_i = (delta_ij - sum_{k < i} M_ik x_k) /
// M_ii (the x_k above row j are zero, so the sum needs no lower limit).
__global__ __launch_bounds__(64) void k_tri_diag_inv(const OpDev* ops, const double* aug, double* minv,
                                                     const int32_t* tri, const double* scale, int* status) {
  const int op = blockIdx.y, b = blockIdx.x;
  if (!tri[op]) return;
  const OpDev o = ops[op];
  const int mp = o.mp;
  if (32 * b >= mp) return;
  const int r0 = 32 * b, W = 2 * mp;
  __shared__ double Mb[32][33];
  __shared__ double Xb[32][33];
  for (int e = threadIdx.x; e < 32 * 32; e += 64) {
    const int r = e / 32, c = e % 32;
    Mb[r][c] = aug[o.sc_aug + (int64_t)(r0 + r) * W + r0 + c];
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j < 32) {
    double x[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      double acc = i == j ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) acc = fma(-Mb[i][k], x[k], acc);
      x[i] = acc / Mb[i][i];
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) Xb[i][j] = x[i];
    const double thresh = (double)mp * DBL_EPSILON * scale[op];
    if (!(fabs(Mb[j][j]) > thresh)) atomicOr(status, 1);
  }
  __syncthreads();
  // the block row of the inverse: the diagonal block and zeros to its right
  // (the blocks to its left come from the doubling GEMMs)
  for (int e = threadIdx.x; e < 32 * (mp - r0); e += 64) {
    const int r = e / (mp - r0), c = r0 + e % (mp - r0);
    minv[o.minv + (int64_t)(r0 + r) * mp + c] = c < r0 + 32 ? Xb[r][c - r0] : 0.0;
  }
}

hipError_t launch_tri_diag_inv(const OpDev* ops, int n_ops, int max_mp, const double* aug, double* minv,
                               const int32_t* tri, const double* scale, int* status, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_diag_inv, dim3(max_mp / 32, n_ops), dim3(64), 0, s, ops, aug, minv, tri, scale, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched FP64 GEMM, C = alpha op(A) op(B) + beta C (row-major), on the FP64
// matrix cores: 64x64 output tile per workgroup, each of the 4 waves owns a
// 32x32 quarter as 2x2 blocks of v_mfma_f64_16x16x4f64. blockIdx.z = job.
// Lane layout of the 16x16x4 FP64 MFMA: A[i=lane%16][k=lane/16],
// B[k=lane/16][j=lane%16], C[i=lane/16+4v][j=lane%16] (register v).
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_f64(const GemmJob* jobs) {
  const GemmJob jb = jobs[blockIdx.z];
  if (jb.gate && *jb.gate == 0) return;
  const int tm = blockIdx.y * 64, tn = blockIdx.x * 64;
  if (tm >= jb.M || tn >= jb.N) return;
  // K in chunks of KT; the next chunk's elements are loaded into registers
  // while the current one is contracted from LDS
  constexpr int KT = 32;
  constexpr int PER = 64 * KT / 256;  // elements of A (and of B) per thread and chunk
  __shared__ double As[64][KT + 1];   // As[i][k] = op(A)(tm+i, k0+k)
  __shared__ double Bs[64][KT + 1];   // Bs[j][k] = op(B)(k0+k, tn+j)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  f64x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // element e of a chunk: (i, kk) of A and (j, kk) of B, consecutive e along
  // the operand's contiguous direction
  auto a_pos = [&](int e, int& i, int& kk) {
    if (jb.transA) {  // A stored K x M: consecutive i contiguous
      i = e % 64;
      kk = e / 64;
    } else {
      i = e / KT;
      kk = e % KT;
    }
  };
  auto b_pos = [&](int e, int& j, int& kk) {
    if (jb.transB) {  // B stored N x K: consecutive k contiguous
      j = e / KT;
      kk = e % KT;
    } else {
      j = e % 64;
      kk = e / 64;
    }
  };
  double ra[PER], rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      int i, j, kk;
      const int e = tid + 256 * t;
      a_pos(e, i, kk);
      const int gi = tm + i, gk = k0 + kk;
      ra[t] = gi < jb.M && gk < jb.K ? (jb.transA ? jb.A[(int64_t)gk * jb.lda + gi] : jb.A[(int64_t)gi * jb.lda + gk])
                                     : 0.0;
      b_pos(e, j, kk);
      const int gj = tn + j, gk2 = k0 + kk;
      rb[t] = gj < jb.N && gk2 < jb.K ? (jb.transB ? jb.B[(int64_t)gj * jb.ldb + gk2] : jb.B[(int64_t)gk2 * jb.ldb + gj])
                                      : 0.0;
    }
  };
  // the K range where both operands of this output tile can be nonzero
  int kb = 0, ke = jb.K;
  if (jb.tri && *jb.tri) {
    if (jb.tri_mode & 1) ke = min(ke, tm + 64);  // op(A)(i, k) = 0 for k > i
    if (jb.tri_mode & 2) kb = max(kb, tm);       // op(A)(i, k) = 0 for k < i
    if (jb.tri_mode & 4) kb = max(kb, tn);       // op(B)(k, j) = 0 for k < j
    if (jb.tri_mode & 8) ke = min(ke, tn + 64);  // op(B)(k, j) = 0 for k > j
    kb = kb / KT * KT;
  }
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += KT) {
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      int i, j, kk;
      const int e = tid + 256 * t;
      a_pos(e, i, kk);
      As[i][kk] = ra[t];
      b_pos(e, j, kk);
      Bs[j][kk] = rb[t];
    }
    __syncthreads();
    if (k0 + KT < ke) load(k0 + KT);
#pragma unroll
    for (int ks = 0; ks < KT; ks += 4) {
      const int kk = ks + (lane >> 4);
      const double a0 = As[wi + (lane & 15)][kk];
      const double a1 = As[wi + 16 + (lane & 15)][kk];
      const double b0 = Bs[wj + (lane & 15)][kk];
      const double b1 = Bs[wj + 16 + (lane & 15)][kk];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 2; ++b) {
      const int gj = tn + wj + b * 16 + (lane & 15);
      for (int v = 0; v < 4; ++v) {
        const int gi = tm + wi + a * 16 + (lane >> 4) + 4 * v;
        if (gi < jb.M && gj < jb.N) {
          double* cp = jb.C + (int64_t)gi * jb.ldc + gj;
          const double r = jb.alpha * acc[a][b][v];
          *cp = jb.beta == 0.0 ? r : r + jb.beta * *cp;
        }
      }
    }
  }
}

hipError_t launch_gemm_f64(const GemmJob* jobs_dev, int n_jobs, int max_m, int max_n,
                           hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  dim3 grid((max_n + 63) / 64, (max_m + 63) / 64, n_jobs);
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, s, jobs_dev);
  return hipGetLastError();
}

// C = alpha A + beta C for each job (blockIdx.y = job); M x N, row-major.
__global__ void k_axpy(const GemmJob* jobs) {
  const GemmJob jb = jobs[blockIdx.y];
  const int n = jb.M * jb.N;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int i = e / jb.N, j = e % jb.N;
    double* cp = jb.C + (int64_t)i * jb.ldc + j;
    const double r = jb.alpha * jb.A[(int64_t)i * jb.lda + j];
    *cp = jb.beta == 0.0 ? r : r + jb.beta * *cp;
  }
}

hipError_t launch_axpy(const GemmJob* jobs_dev, int n_jobs, int max_m, int max_n,
                       hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  int bx = (max_m * max_n + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_axpy, dim3(bx, n_jobs), dim3(256), 0, s, jobs_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cast of the powers to the compute type and of the small matrices to the
// state type. FP64 -> bfloat16 is rounded once, to nearest even, straight
// from the FP64 value (no intermediate FP32 rounding) in the FP32 normal
// range; below it the value goes through FP32 first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f64_to_bf16_bits(double d) {
  const uint64_t bits = (uint64_t)__double_as_longlong(d);
  const uint64_t sign = bits & 0x8000000000000000ull;
  uint64_t mag = bits & 0x7fffffffffffffffull;
  if (mag > 0x7ff0000000000000ull) return (uint16_t)((sign >> 48) | 0x7fc0u);  // NaN
  if (mag < (uint64_t)(1023 - 126) << 52) {  // below FP32 normal range
    const uint32_t u = __float_as_uint((float)d);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
  }
  // keep 7 fraction bits: drop the low 45 bits with round-to-nearest-even
  const uint64_t lsb = (mag >> 45) & 1ull;
  mag += (1ull << 44) - 1ull + lsb;
  mag &= ~((1ull << 45) - 1ull);
  const float f = (float)__longlong_as_double((long long)(sign | mag));  // exact (or inf)
  return (uint16_t)(__float_as_uint(f) >> 16);
}

__global__ void k_pack_powers(const OpDev* ops, const double* pw, void* pc, int ct, int want_t) {
  const OpDev o = ops[blockIdx.y];
  const int mp = o.mp;
  const int64_t n = (int64_t)(o.N + 1) * mp * mp;
  const int64_t mm = (int64_t)mp * mp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = pw[o.pw + e];
    const int64_t kslot = e / mm, rc = e % mm;
    const int64_t r = rc / mp, c = rc % mp;
    const int64_t et = kslot * mm + c * mp + r;  // transposed position
    if (ct == DT_BF16) {
      const uint16_t b = f64_to_bf16_bits(v);
      ((uint16_t*)pc)[o.pc + e] = b;
      if (want_t) ((uint16_t*)pc)[o.pct + et] = b;
    } else if (ct == DT_F32) {
      const float f = (float)v;
      ((float*)pc)[o.pc + e] = f;
      if (want_t) ((float*)pc)[o.pct + et] = f;
    } else {
      ((double*)pc)[o.pc + e] = v;
      if (want_t) ((double*)pc)[o.pct + et] = v;
    }
  }
}

__global__ void k_pack_krylov(const OpDev* ops, const double* kw, void* kc, int ct) {
  const OpDev o = ops[blockIdx.y];
  auto cast = [&](int64_t from, int64_t to, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
      const double v = kw[from + e];
      if (ct == DT_BF16)
        ((uint16_t*)kc)[to + e] = f64_to_bf16_bits(v);
      else if (ct == DT_F32)
        ((float*)kc)[to + e] = (float)v;
      else
        ((double*)kc)[to + e] = v;
    }
  };
  if (o.kw >= 0) cast(o.kw, o.kc, (int64_t)o.mp * o.kst);  // K_j
  if (o.cpl >= 0) cast(o.cpw, o.cpc, (int64_t)16 * o.mp);  // C P_l of the tail pair
}

hipError_t launch_pack_krylov(const OpDev* ops, int n_ops, const double* kw, void* kc, int ct,
                              int max_mp, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  int blocks = (max_mp * max_mp + 255) / 256;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(k_pack_krylov, dim3(blocks, n_ops), dim3(256), 0, s, ops, kw, kc, ct);
  return hipGetLastError();
}

// G_j (16 x mp FP64 blocks, j < 2^fold_s) into operand order: chunk (j, t,
// lane) holds G_j[lane % 16][32 t + 8 (lane / 16) .. + 7], eight values of the
// compute type (BF16 only).
__global__ void k_pack_fold(const OpDev* ops, const double* gw, uint16_t* gc) {
  const OpDev o = ops[blockIdx.y];
  if (o.fold_s <= 0) return;
  const int mp = o.mp, ks = mp / 32;
  // elements: 2^s G_j of 16 x mp, or half as many paired operands
  const int64_t n = (((int64_t)1 << o.fold_s) * 16 * mp) >> (o.fold_paired ? 1 : 0);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)(e & 7);
    const int64_t chunk = e >> 3;
    const int lane = (int)(chunk & 63);
    const int64_t jt = chunk >> 6;
    const int t = (int)(jt % ks), j = (int)(jt / ks);
    // operand j: G_j, or G_{2j} (rows 0..7) over G_{2j+1} (rows 8..15)
    const int row = o.fold_paired ? (2 * j + ((lane & 15) >> 3)) * 16 + (lane & 7) : j * 16 + (lane & 15);
    const int col = 32 * t + 8 * (lane >> 4) + v;
    gc[o.fold_gc + e] = f64_to_bf16_bits(gw[o.fold_gw + (int64_t)row * mp + col]);
  }
}

hipError_t launch_pack_fold(const OpDev* ops, int n_ops, const double* gw, void* gc, int ct, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  if (ct != DT_BF16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_fold, dim3(128, n_ops), dim3(256), 0, s, ops, gw, (uint16_t*)gc);
  return hipGetLastError();
}

template <typename X>
__global__ void k_pack_small(const OpDev* ops, const OpSrc* src, const double* bbar, X* sm) {
  const OpDev o = ops[blockIdx.y];
  const OpSrc sp = src[blockIdx.y];
  const int mp = o.mp, m = o.m, p = o.p, q = o.q;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  for (int e = tid; e < mp * p; e += nth) {  // Bbar (mp x p) and Bbar^T (p x mp)
    const int r = e / p, c = e % p;
    const X v = (X)bbar[o.bbar + e];
    sm[o.bin + e] = v;
    sm[o.bt + (int64_t)c * mp + r] = v;
  }
  for (int e = tid; e < q * mp; e += nth) {  // C (q x mp) and C^T (mp x q)
    const int r = e / mp, c = e % mp;
    const X v = c < m ? (X)sp.C[(int64_t)r * m + c] : (X)0;
    sm[o.cout + e] = v;
    sm[o.ct + (int64_t)c * q + r] = v;
  }
  for (int e = tid; e < q * p; e += nth) {  // D (q x p) and D^T (p x q)
    const int r = e / p, c = e % p;
    const X v = (X)sp.D[(int64_t)r * p + c];
    sm[o.dmat + e] = v;
    sm[o.dt + (int64_t)c * q + r] = v;
  }
}

hipError_t launch_pack(const OpDev* ops, int n_ops, const OpSrc* src, const double* pw,
                       const double* bbar, void* pc, int ct, int want_t, void* small,
                       int state_is_f64, int max_mp, int max_N, hipStream_t s) {
  if (n_ops <= 0) return hipSuccess;
  const int64_t n = (int64_t)(max_N + 1) * max_mp * max_mp;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_pack_powers, dim3(blocks, n_ops), dim3(256), 0, s, ops, pw, pc, ct,
                     want_t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (state_is_f64)
    hipLaunchKernelGGL(k_pack_small<double>, dim3(8, n_ops), dim3(256), 0, s, ops, src, bbar,
                       (double*)small);
  else
    hipLaunchKernelGGL(k_pack_small<float>, dim3(8, n_ops), dim3(256), 0, s, ops, src, bbar,
                       (float*)small);
  return hipGetLastError();
}

}  // namespace ssmc
