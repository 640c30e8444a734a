// Initial state x_{-1} for the forward apply.
//
// Unrolling eq. (1.2) from a nonzero x_{-1} gives x_l = Abar^(l+1) x_{-1} +
// sum_{j<=l} Abar^j Bbar u_{l-j}: the initial state acts as one more input,
// Abar x_{-1}, at row 0. The first pass of an apply leaves the state after a
// sequence's first kry stages in buffer kry % 2 (kry = 0: V^(0) = Bbar u
// itself, in buffer 0); those stages have added every lag below 2^kry, so the
// extra input shows there as Abar^(l+1) x_{-1} in rows l < 2^kry, and the
// remaining stages, linear in the state, carry it on like the rest. This pass
// adds those rows: one workgroup per sequence forms w_0 = Abar x0, w_{l+1} =
// Abar w_l in FP64 (thread e owns entry e) and adds w_l to row l of the state.
// Where the first pass already ran every stage of a sequence and formed its
// output (kry = last + 1), no later pass reads that state, so the free
// response goes straight into the output instead: y_l += C w_l, y = C x + D u
// being linear in the state (and, when the plan keeps final states, into the
// state rows as well).
#include "ssm_internal.h"

namespace ssmc {

template <typename X>
__global__ __launch_bounds__(256) void k_inject_x0(const SeqDev* seqs, const OpDev* ops, const double* pw,
                                                   const X* x0, int mp_class, X* buf0, X* buf1,
                                                   const X* small, X* y, int keep_state) {
  __shared__ double w[2][256];
  const int s = blockIdx.x;
  const SeqDev sq = seqs[s];
  const OpDev o = ops[sq.op];
  if (o.mp != mp_class) return;  // (uniform: the whole workgroup leaves)
  // x0 holds the states of the sequences in order, m of each
  int64_t off = 0;
  for (int i = 0; i < s; ++i) off += ops[seqs[i].op].m;
  const int m = o.m, mp = o.mp, e = threadIdx.x;
  const int64_t R = sq.L < ((int64_t)1 << sq.kry) ? sq.L : ((int64_t)1 << sq.kry);
  const double* A = pw + o.pw;  // Abar, mp x mp, zero padded
  X* xb = (sq.kry & 1 ? buf1 : buf0) + sq.x_off;
  // (kry = 0 never ends a sequence: its stages and output are still to run)
  const bool to_y = sq.kry > 0 && sq.kry == sq.last + 1;
  const X* cm = small + o.cout;  // C, q x mp, in the state type
  X* yb = y + sq.y_off;
  w[0][e] = e < m ? (double)x0[off + e] : 0.0;
  __syncthreads();
  for (int64_t l = 0; l < R; ++l) {
    const double* src = w[l & 1];
    double acc = 0.0;
    if (e < m) {
      const double* row = A + (int64_t)e * mp;
      for (int k = 0; k < m; ++k) acc = fma(row[k], src[k], acc);
      if (!to_y || keep_state) {
        X* dst = xb + l * mp + e;
        *dst = (X)((double)*dst + acc);
      }
    }
    w[(l + 1) & 1][e] = acc;
    __syncthreads();
    if (to_y && e < sq.q) {  // w_l is complete in w[(l + 1) & 1]
      const double* wl = w[(l + 1) & 1];
      double a = 0.0;
      for (int k = 0; k < m; ++k) a = fma((double)cm[(int64_t)e * mp + k], wl[k], a);
      X* dst = yb + l * sq.q + e;
      *dst = (X)((double)*dst + a);
    }
  }
}

hipError_t launch_inject_x0(int mp_class, bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops,
                            const double* pw, const void* x0, void* buf0, void* buf1, const void* small,
                            void* y, bool keep_state, hipStream_t st) {
  if (n_seq <= 0) return hipSuccess;
  if (mp_class > 256) return hipErrorInvalidValue;
  if (f64)
    hipLaunchKernelGGL(k_inject_x0<double>, dim3(n_seq), dim3(256), 0, st, seqs, ops, pw,
                       static_cast<const double*>(x0), mp_class, static_cast<double*>(buf0),
                       static_cast<double*>(buf1), static_cast<const double*>(small), static_cast<double*>(y),
                       (int)keep_state);
  else
    hipLaunchKernelGGL(k_inject_x0<float>, dim3(n_seq), dim3(256), 0, st, seqs, ops, pw,
                       static_cast<const float*>(x0), mp_class, static_cast<float*>(buf0),
                       static_cast<float*>(buf1), static_cast<const float*>(small), static_cast<float*>(y),
                       (int)keep_state);
  return hipGetLastError();
}

// The backward from an initial state recomputes the forward from V^(0) =
// Bbar u: the initial state is the input Abar x_{-1} added to row 0 of V^(0)
// (one workgroup per sequence, FP64 matvec).
template <typename X>
__global__ __launch_bounds__(256) void k_input_x0(const SeqDev* seqs, const OpDev* ops, const double* pw,
                                                  const X* x0, int mp_class, X* v0) {
  const int s = blockIdx.x;
  const SeqDev sq = seqs[s];
  const OpDev o = ops[sq.op];
  if (o.mp != mp_class) return;
  int64_t off = 0;
  for (int i = 0; i < s; ++i) off += ops[seqs[i].op].m;
  __shared__ double xs[256];
  const int e = threadIdx.x, m = o.m;
  xs[e] = e < m ? (double)x0[off + e] : 0.0;
  __syncthreads();
  if (e < m) {
    const double* row = pw + o.pw + (int64_t)e * o.mp;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc = fma(row[k], xs[k], acc);
    X* dst = v0 + sq.x_off + e;
    *dst = (X)((double)*dst + acc);
  }
}

hipError_t launch_input_x0(int mp_class, bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops,
                           const double* pw, const void* x0, void* v0, hipStream_t st) {
  if (n_seq <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_input_x0<double>, dim3(n_seq), dim3(256), 0, st, seqs, ops, pw,
                       static_cast<const double*>(x0), mp_class, static_cast<double*>(v0));
  else
    hipLaunchKernelGGL(k_input_x0<float>, dim3(n_seq), dim3(256), 0, st, seqs, ops, pw,
                       static_cast<const float*>(x0), mp_class, static_cast<float*>(v0));
  return hipGetLastError();
}

// Gradients of the initial state: with g = dL/dV^(0) (the adjoint cascade's
// result, row 0 of every sequence in g0), dL/dx_{-1} = Abar^T g_0 and the
// direct part of dL/dAbar is g_0 x_{-1}^T, added to dL/dP_0 before the
// squaring adjoint. One workgroup per operator walks its sequences in order,
// so the sum over sequences sharing the operator has a fixed order; thread e
// owns row e (FP64).
template <typename X>
__global__ __launch_bounds__(256) void k_x0_grads(const SeqDev* seqs, int n_seq, const OpDev* ops,
                                                  const double* pw, const X* x0, const X* g0, X* dx0,
                                                  double* G) {
  const int op = blockIdx.x;
  const OpDev o = ops[op];
  const int e = threadIdx.x, m = o.m, mp = o.mp;
  __shared__ double gs[256], xs[256];
  int64_t off = 0;
  for (int s = 0; s < n_seq; ++s) {
    const SeqDev sq = seqs[s];
    const int ms = ops[sq.op].m;
    if (sq.op == op) {
      __syncthreads();
      gs[e] = e < m ? (double)g0[sq.x_off + e] : 0.0;
      xs[e] = e < m && x0 ? (double)x0[off + e] : 0.0;
      __syncthreads();
      if (e < m) {
        if (dx0) {
          double acc = 0.0;
          for (int k = 0; k < m; ++k) acc = fma(pw[o.pw + (int64_t)k * mp + e], gs[k], acc);
          dx0[off + e] = (X)acc;
        }
        if (G) {
          double* row = G + o.g_dp + (int64_t)e * mp;
          for (int k = 0; k < m; ++k) row[k] = fma(gs[e], xs[k], row[k]);
        }
      }
    }
    off += ms;
  }
}

hipError_t launch_x0_grads(bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops, int n_ops, const double* pw,
                           const void* x0, const void* g0, void* dx0, double* G, hipStream_t st) {
  if (n_ops <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_x0_grads<double>, dim3(n_ops), dim3(256), 0, st, seqs, n_seq, ops, pw,
                       static_cast<const double*>(x0), static_cast<const double*>(g0), static_cast<double*>(dx0), G);
  else
    hipLaunchKernelGGL(k_x0_grads<float>, dim3(n_ops), dim3(256), 0, st, seqs, n_seq, ops, pw,
                       static_cast<const float*>(x0), static_cast<const float*>(g0), static_cast<float*>(dx0), G);
  return hipGetLastError();
}

// The state of a sequence's last row, x_{L-1}, for the next chunk of a
// stream. With final states kept, the epilogue of a sequence's last stage
// (or of its input pass, when that pass runs every stage) has stored the
// state after that stage, and the state after stage k lives in buffer
// (k + 1) mod 2 (V^(0) = Bbar u, "after stage -1", in buffer 0). One
// workgroup per sequence copies row L - 1 (its m entries) into x_last.
template <typename X>
__global__ __launch_bounds__(256) void k_gather_last(const SeqDev* seqs, const OpDev* ops, const X* buf0,
                                                     const X* buf1, X* x_last) {
  const int s = blockIdx.x;
  const SeqDev sq = seqs[s];
  const OpDev o = ops[sq.op];
  int64_t off = 0;
  for (int i = 0; i < s; ++i) off += ops[seqs[i].op].m;
  const X* src = ((sq.last + 1) & 1 ? buf1 : buf0) + sq.x_off + (sq.L - 1) * o.mp;
  for (int e = threadIdx.x; e < o.m; e += 256) x_last[off + e] = src[e];
}

hipError_t launch_gather_last(bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops, const void* buf0,
                              const void* buf1, void* x_last, hipStream_t st) {
  if (n_seq <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_gather_last<double>, dim3(n_seq), dim3(256), 0, st, seqs, ops,
                       static_cast<const double*>(buf0), static_cast<const double*>(buf1),
                       static_cast<double*>(x_last));
  else
    hipLaunchKernelGGL(k_gather_last<float>, dim3(n_seq), dim3(256), 0, st, seqs, ops,
                       static_cast<const float*>(buf0), static_cast<const float*>(buf1),
                       static_cast<float*>(x_last));
  return hipGetLastError();
}

}  // namespace ssmc
