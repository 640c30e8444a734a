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
