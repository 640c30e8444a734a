// Host side of the C ABI declared in include/ssm_cascade.h: the entry points,
// device tables and the launch sequences of prepare / apply / recursion /
// backward and their graphs (the plan itself is built in plan.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ssm_cascade.h"
#include "plan.h"
#include "ssm_internal.h"
#include "plr.h"

using namespace ssmc;
using namespace ssmc::host;

namespace {

#define HIP_TRY(expr, what)                    \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

// Records an event pair around a launch when timing is on.
struct TimedLaunch {
  ssm_plan_s& P;
  hipStream_t s;
  int kind;
  bool on;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(ssm_plan_s& P_, hipStream_t s_, int kind_, bool allowed = true)
      : P(P_), s(s_), kind(kind_), on(P_.timing && allowed) {
    if (on) {
      a = take();
      b = take();
      (void)hipEventRecord(a, s);
    }
  }
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!P.event_pool.empty()) {
      e = P.event_pool.back();
      P.event_pool.pop_back();
    } else {
      (void)hipEventCreate(&e);
    }
    return e;
  }
  void done() {
    if (on) {
      (void)hipEventRecord(b, s);
      P.trec.push_back(TimingRec{kind, a, b});
    }
  }
};

ssm_status check_io(const ssm_plan_s& P, const void* u, ssm_dtype u_dtype, size_t u_numel,
                    const void* y, size_t y_numel, const char* yname) {
  if (!u) return fail(SSM_E_INVALID, "u is NULL");
  if (!y) return fail(SSM_E_INVALID, "%s is NULL", yname);
  if (P.state_f64) {
    if (u_dtype != SSM_F64) return fail(SSM_E_INVALID, "an F64 plan takes F64 input");
  } else if (u_dtype != SSM_F32 && u_dtype != SSM_BF16) {
    return fail(SSM_E_INVALID, "an F32/BF16 plan takes F32 or BF16 input");
  }
  for (int i = 0; i < P.n_seq; ++i) {
    const SeqDev& s = P.seqs[i];
    if ((size_t)s.u_off + (size_t)s.L * s.p > u_numel)
      return fail(SSM_E_INVALID, "seq %d: u block [%lld, +%lld) exceeds u_numel %zu", i,
                  (long long)s.u_off, (long long)(s.L * s.p), u_numel);
    if ((size_t)s.y_off + (size_t)s.L * s.q > y_numel)
      return fail(SSM_E_INVALID, "seq %d: %s block [%lld, +%lld) exceeds numel %zu", i, yname,
                  (long long)s.y_off, (long long)(s.L * s.q), y_numel);
  }
  return SSM_OK;
}

// One per-stage launch of class c at stage prm.k: the chain kernel where the
// plan has units for this stage, else the resident-power kernel where the plan
// uses it and it can apply this stage, the tiled one otherwise. Where the
// resident kernels split the state rows between workgroups (FP32, padded m
// 256) they have no output epilogue: a last stage then runs lean and
// k_output_proj forms the output from the rows it stored.
hipError_t launch_stage_any(const ssm_plan_s& P, int c, StageParams prm, hipStream_t stream) {
  const int mp = kClassMp[c];
  const int k = prm.k;
  const bool splits = res_splits_rows(mp, P.compute);
  const bool final_here = (prm.flags & SF_EPILOGUE) &&
                          (prm.adjoint ? k == 0 : (k < (int)P.class_final[c].size() &&
                                                   P.class_final[c][k] > 0));
  // lean stage + k_output_proj: every sequence of the class within that
  // kernel's sizes and 32-bit row offsets, and no final-state copy asked for
  bool proj = splits && final_here && !prm.xfinal && !(prm.flags & SF_NOUPDATE) &&
              P.stage_kernel != SSM_STAGE_TILED;
  for (int i = 0; proj && i < P.n_seq; ++i) {
    const SeqDev& sq = P.seqs[i];
    if (P.ops[sq.op].mp != mp) continue;
    proj = output_proj_supported(mp, P.compute, prm.adjoint ? sq.p : sq.q, prm.adjoint ? sq.q : sq.p) &&
           sq.L * (int64_t)mp * 4 < ((int64_t)1 << 31);
  }
  const ResRange* rg = reinterpret_cast<const ResRange*>(P.ws + P.r_meta.off + P.m_ranges) +
                       P.class_range_start[c];
  StageParams lean = prm;
  lean.flags &= ~(SF_EPILOGUE | SF_STORE_AT_EPI);
  if (k < (int)P.chain_count[c].size() && P.chain_count[c][k] > 0) {
    const ChainUnit* un = reinterpret_cast<const ChainUnit*>(P.ws + P.r_meta.off + P.m_chain) +
                          P.chain_start[c][k];
    const bool tail = prm.adjoint ? k == 0 : P.class_final[c][k] > 0;
    const int tri = P.compute == DT_F32 && P.class_lower[c] ? (prm.adjoint ? 2 : 1) : 0;
    if (!(tail && splits))
      return launch_stage_chain(mp, P.compute, prm, un, P.chain_count[c][k], tail, tri, stream);
    if (proj) {
      hipError_t e = launch_stage_chain(mp, P.compute, lean, un, P.chain_count[c][k], false, tri, stream);
      if (e != hipSuccess) return e;
      return launch_output_proj(mp, prm, rg, P.class_range_active[c][k], stream);
    }
  }
  if (P.stage_kernel != SSM_STAGE_TILED && res_supported(mp, P.compute)) {
    if (!(final_here && splits))
      return launch_stage_res(mp, P.compute, prm, rg, P.class_range_active[c][k], stream);
    if (proj) {
      hipError_t e = launch_stage_res(mp, P.compute, lean, rg, P.class_range_active[c][k], stream);
      if (e != hipSuccess) return e;
      return launch_output_proj(mp, prm, rg, P.class_range_active[c][k], stream);
    }
  }
  return launch_stage(mp, P.compute, P.class_bm[c], prm, stream);
}

StageParams base_params(const ssm_plan_s& P, int c) {
  StageParams prm{};
  prm.tiles = reinterpret_cast<const Tile*>(P.ws + P.r_meta.off + P.m_tiles) +
              P.class_tile_start[c];
  prm.seqs = reinterpret_cast<const SeqDev*>(P.ws + P.r_meta.off + P.m_seqs);
  prm.ops = reinterpret_cast<const OpDev*>(P.ws + P.r_meta.off + P.m_ops);
  prm.P = P.ws + P.r_pc.off;
  prm.small = P.ws + P.r_small.off;
  return prm;
}

// Jobs of the adjoint of the exponential discretization, run by the backward
// after the squaring adjoint has left dL/dAbar in g_dp (k = 0) and dL/dBbar in
// g_dbb. For F = exp(E), the adjoint of dF = L(E, dE) is G -> L(E^T, G), the
// upper-right block of exp([[E^T, G], [0, E^T]]); with G = [[dL/dAbar,
// dL/dBbar], [0, 0]] and E = delta [[A, B], [0, 0]], dL/dA = delta L[:m, :m]
// and dL/dB = delta L[:m, m:]. The block upper-triangular exponential is
// carried as its pair of blocks (D, F): the same scaling by 2^-s as the
// forward (X = E / 2^s is still in the scratch, used transposed), Horner steps
// (D, F) <- (I + X^T D / k, (X^T F + Y D) / k) with Y = G / 2^s, and s
// squarings (D, F) <- (D D, D F + F D).
ssm_status zoh_adjoint_jobs(ssm_plan_s& P) {
  double* zs = P.at<double>(P.r_zoh);
  double* G = P.at<double>(P.r_g);
  const double* I = zs + P.z_id;
  const int nid = P.z_nid;
  P.zbjobs.clear();
  P.zbgroups.clear();
  P.zbdims.clear();
  P.zbkind.clear();
  std::vector<GemmJob>& J = P.zbjobs;
  const size_t nops = P.ops.size();
  std::vector<double*> Sd(nops), Td(nops), Sf(nops), Tf(nops), Y(nops), X(nops);
  for (size_t i = 0; i < nops; ++i) {
    const OpDev& o = P.ops[i];
    const int64_t nn = (int64_t)o.zn * o.zn;
    X[i] = zs + o.zx;
    Sd[i] = X[i] + nn;
    Td[i] = X[i] + 2 * nn;
    Sf[i] = X[i] + 3 * nn;
    Tf[i] = X[i] + 4 * nn;
    Y[i] = X[i] + 5 * nn;
  }
  auto group = [&](int kind, auto&& fill) {
    const int start = (int)J.size();
    int mx = 0, mn = 0;
    for (size_t i = 0; i < nops; ++i) fill(i);
    for (size_t j = start; j < J.size(); ++j) {
      mx = std::max(mx, J[j].M);
      mn = std::max(mn, J[j].N);
    }
    if ((int)J.size() > start) {
      P.zbgroups.push_back({start, (int)J.size() - start});
      P.zbdims.push_back({mx, mn});
      P.zbkind.push_back(kind);
    }
  };
  group(1, [&](size_t i) {  // Y = 0, D = I, F = 0 (zeros as 0 times the identity)
    const OpDev& o = P.ops[i];
    J.push_back(GemmJob{I, nullptr, Y[i], o.zn, o.zn, 0, nid, 0, o.zn, 0, 0, 0.0, 0.0});
    J.push_back(GemmJob{I, nullptr, Sd[i], o.zn, o.zn, 0, nid, 0, o.zn, 0, 0, 1.0, 0.0});
    J.push_back(GemmJob{I, nullptr, Sf[i], o.zn, o.zn, 0, nid, 0, o.zn, 0, 0, 0.0, 0.0});
  });
  group(1, [&](size_t i) {  // Y = [[dL/dAbar, dL/dBbar], [0, 0]] / 2^s
    const OpDev& o = P.ops[i];
    const double sc = std::ldexp(1.0, -o.zsq);
    J.push_back(GemmJob{G + o.g_dp, nullptr, Y[i], o.m, o.m, 0, o.mp, 0, o.zn, 0, 0, sc, 0.0});
    J.push_back(GemmJob{G + o.g_dbb, nullptr, Y[i] + o.m, o.m, o.p, 0, o.p, 0, o.zn, 0, 0, sc, 0.0});
  });
  for (int k = kZohTaylor; k >= 1; --k) {
    group(1, [&](size_t i) {  // T_D = I
      const OpDev& o = P.ops[i];
      J.push_back(GemmJob{I, nullptr, Td[i], o.zn, o.zn, 0, nid, 0, o.zn, 0, 0, 1.0, 0.0});
    });
    group(0, [&](size_t i) {  // T_D = X^T S_D / k + T_D;  T_F = X^T S_F / k
      const OpDev& o = P.ops[i];
      J.push_back(GemmJob{X[i], Sd[i], Td[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 1, 0, 1.0 / k, 1.0});
      J.push_back(GemmJob{X[i], Sf[i], Tf[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 1, 0, 1.0 / k, 0.0});
    });
    group(0, [&](size_t i) {  // T_F = Y S_D / k + T_F
      const OpDev& o = P.ops[i];
      J.push_back(GemmJob{Y[i], Sd[i], Tf[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 0, 0, 1.0 / k, 1.0});
    });
    for (size_t i = 0; i < nops; ++i) {
      std::swap(Sd[i], Td[i]);
      std::swap(Sf[i], Tf[i]);
    }
  }
  int max_sq = 0;
  for (const OpDev& o : P.ops) max_sq = std::max(max_sq, o.zsq);
  for (int t = 0; t < max_sq; ++t) {
    group(0, [&](size_t i) {  // T_D = S_D S_D;  T_F = S_D S_F
      const OpDev& o = P.ops[i];
      if (o.zsq <= t) return;
      J.push_back(GemmJob{Sd[i], Sd[i], Td[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 0, 0, 1.0, 0.0});
      J.push_back(GemmJob{Sd[i], Sf[i], Tf[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 0, 0, 1.0, 0.0});
    });
    group(0, [&](size_t i) {  // T_F = S_F S_D + T_F
      const OpDev& o = P.ops[i];
      if (o.zsq <= t) return;
      J.push_back(GemmJob{Sf[i], Sd[i], Tf[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 0, 0, 1.0, 1.0});
    });
    for (size_t i = 0; i < nops; ++i)
      if (P.ops[i].zsq > t) {
        std::swap(Sd[i], Td[i]);
        std::swap(Sf[i], Tf[i]);
      }
  }
  group(1, [&](size_t i) {  // dL/dA = delta F[:m, :m], dL/dB = delta F[:m, m:]
    const OpDev& o = P.ops[i];
    J.push_back(GemmJob{Sf[i], nullptr, G + o.g_da, o.m, o.m, 0, o.zn, 0, o.mp, 0, 0, o.delta, 0.0});
    J.push_back(GemmJob{Sf[i] + o.m, nullptr, G + o.g_db, o.m, o.p, 0, o.zn, 0, o.p, 0, 0, o.delta, 0.0});
  });
  if (J.size() > P.zb_cap) return fail(SSM_E_INVALID, "exponential adjoint job table overflow");
  return SSM_OK;
}

// Exponential discretization (§5) of every operator: exp(E), E = delta [[A,
// B], [0, 0]], whose blocks are Abar = exp(delta A) and Bbar = int_0^delta
// exp(sA) ds B. The norms of E come back to the host, which fixes per operator
// the squarings s with |E|_1 / 2^s <= 1/2; then X = E / 2^s, the Taylor
// polynomial by Horner steps S <- I + X S / k (k = kZohTaylor .. 1), s
// squarings, and the copies of the blocks into P_0 and Bbar, each step one
// launch over all operators (FP64 GEMM and axpy jobs).
ssm_status zoh_discretize(ssm_plan_s& P, const OpDev* ops_d, const OpSrc* src_d, hipStream_t stream) {
  double* zs = P.at<double>(P.r_zoh);
  double* pw = P.at<double>(P.r_pw);
  double* bbar = P.at<double>(P.r_bbar);
  int max_n = 0;
  for (const OpDev& o : P.ops) max_n = std::max(max_n, o.zn);
  hipError_t e = launch_zoh_setup(ops_d, P.n_ops, src_d, zs, zs + P.z_id, P.z_nid, zs + P.z_norm, pw, bbar,
                                  max_n, stream);
  if (e != hipSuccess) return hip_fail(e, "exponential setup launch");
  std::vector<double> norms(P.ops.size());
  e = hipMemcpyAsync(norms.data(), zs + P.z_norm, sizeof(double) * norms.size(), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "norm read");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "norm synchronization");
  for (size_t i = 0; i < P.ops.size(); ++i) {
    const double nv = norms[i];
    if (!std::isfinite(nv)) return fail(SSM_E_NUMERIC, "operator %zu: delta [A B] has a non-finite norm", i);
    int sq = 0;
    while (sq <= kZohMaxSq && std::ldexp(nv, -sq) > 0.5) ++sq;
    if (sq > kZohMaxSq)
      return fail(SSM_E_NUMERIC, "operator %zu: |delta [A B]|_1 = %g needs more than %d squarings", i, nv,
                  kZohMaxSq);
    P.ops[i].zsq = sq;
  }
  // jobs (X, S, T: the three scratch matrices of an operator; S and T swap)
  std::vector<GemmJob> J;
  std::vector<std::pair<int, int>> groups, dims;
  std::vector<int> kinds;
  const double* I = zs + P.z_id;
  const int nid = P.z_nid;
  std::vector<double*> S(P.ops.size()), T(P.ops.size());
  auto group = [&](int kind, auto&& fill) {
    const int start = (int)J.size();
    int mx = 0, mn = 0;
    for (size_t i = 0; i < P.ops.size(); ++i) {
      const size_t before = J.size();
      fill(i);
      for (size_t j = before; j < J.size(); ++j) {
        mx = std::max(mx, J[j].M);
        mn = std::max(mn, J[j].N);
      }
    }
    if ((int)J.size() > start) {
      groups.push_back({start, (int)J.size() - start});
      dims.push_back({mx, mn});
      kinds.push_back(kind);
    }
  };
  for (size_t i = 0; i < P.ops.size(); ++i) {
    const OpDev& o = P.ops[i];
    const int64_t nn = (int64_t)o.zn * o.zn;
    S[i] = zs + o.zx + nn;
    T[i] = zs + o.zx + 2 * nn;
  }
  group(1, [&](size_t i) {  // X = E / 2^s;  S = I
    const OpDev& o = P.ops[i];
    double* X = zs + o.zx;
    J.push_back(GemmJob{X, nullptr, X, o.zn, o.zn, 0, o.zn, 0, o.zn, 0, 0, std::ldexp(1.0, -o.zsq), 0.0});
    J.push_back(GemmJob{I, nullptr, S[i], o.zn, o.zn, 0, nid, 0, o.zn, 0, 0, 1.0, 0.0});
  });
  for (int k = kZohTaylor; k >= 1; --k) {
    group(1, [&](size_t i) {  // T = I
      const OpDev& o = P.ops[i];
      J.push_back(GemmJob{I, nullptr, T[i], o.zn, o.zn, 0, nid, 0, o.zn, 0, 0, 1.0, 0.0});
    });
    group(0, [&](size_t i) {  // T = X S / k + T
      const OpDev& o = P.ops[i];
      J.push_back(GemmJob{zs + o.zx, S[i], T[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 0, 0, 1.0 / k, 1.0});
    });
    for (size_t i = 0; i < P.ops.size(); ++i) std::swap(S[i], T[i]);
  }
  int max_sq = 0;
  for (const OpDev& o : P.ops) max_sq = std::max(max_sq, o.zsq);
  for (int t = 0; t < max_sq; ++t) {
    group(0, [&](size_t i) {  // T = S S
      const OpDev& o = P.ops[i];
      if (o.zsq <= t) return;
      J.push_back(GemmJob{S[i], S[i], T[i], o.zn, o.zn, o.zn, o.zn, o.zn, o.zn, 0, 0, 1.0, 0.0});
    });
    for (size_t i = 0; i < P.ops.size(); ++i)
      if (P.ops[i].zsq > t) std::swap(S[i], T[i]);
  }
  group(1, [&](size_t i) {  // P_0 = exp(E)[:m, :m], Bbar = exp(E)[:m, m:]
    const OpDev& o = P.ops[i];
    J.push_back(GemmJob{S[i], nullptr, pw + o.pw, o.m, o.m, 0, o.zn, 0, o.mp, 0, 0, 1.0, 0.0});
    J.push_back(GemmJob{S[i] + o.m, nullptr, bbar + o.bbar, o.m, o.p, 0, o.zn, 0, o.p, 0, 0, 1.0, 0.0});
  });
  if (J.size() > P.z_cap) return fail(SSM_E_INVALID, "exponential job table overflow");
  if (P.with_backward) {
    const ssm_status bs = zoh_adjoint_jobs(P);
    if (bs != SSM_OK) return bs;
  }
  unsigned char* meta = P.ws + P.r_meta.off;
  std::memcpy(P.meta_host.data() + P.m_zjobs, J.data(), sizeof(GemmJob) * J.size());
  e = hipMemcpyAsync(meta + P.m_zjobs, P.meta_host.data() + P.m_zjobs, sizeof(GemmJob) * J.size(),
                     hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "upload of the exponential jobs");
  // the squarings chosen above, for the operator table on the device
  e = hipMemcpyAsync(meta + P.m_ops, P.ops.data(), sizeof(OpDev) * P.ops.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "upload of the operator table");
  if (!P.zbjobs.empty()) {
    std::memcpy(P.meta_host.data() + P.m_zbjobs, P.zbjobs.data(), sizeof(GemmJob) * P.zbjobs.size());
    e = hipMemcpyAsync(meta + P.m_zbjobs, P.meta_host.data() + P.m_zbjobs, sizeof(GemmJob) * P.zbjobs.size(),
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "upload of the exponential adjoint jobs");
  }
  const GemmJob* jd = reinterpret_cast<const GemmJob*>(meta + P.m_zjobs);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const auto& gr = groups[gi];
    e = kinds[gi] == 1 ? launch_axpy(jd + gr.first, gr.second, dims[gi].first, dims[gi].second, stream)
                       : launch_gemm_f64(jd + gr.first, gr.second, dims[gi].first, dims[gi].second, stream);
    if (e != hipSuccess) return hip_fail(e, "exponential launch");
  }
  return SSM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ssm_status_string(ssm_status s) {
  switch (s) {
    case SSM_OK: return "SSM_OK";
    case SSM_E_INVALID: return "SSM_E_INVALID: invalid argument";
    case SSM_E_UNSUPPORTED: return "SSM_E_UNSUPPORTED: not supported";
    case SSM_E_WORKSPACE: return "SSM_E_WORKSPACE: workspace too small";
    case SSM_E_HIP: return "SSM_E_HIP: HIP runtime error";
    case SSM_E_NOT_PREPARED: return "SSM_E_NOT_PREPARED: plan missing or lacks what is needed";
    case SSM_E_NUMERIC: return "SSM_E_NUMERIC: singular discretization matrix";
  }
  return "unknown ssm_status";
}

const char* ssm_last_error(void) { return g_last_error.c_str(); }

size_t ssm_cascade_workspace_bytes(const ssm_seq_desc* seqs, int32_t n_seq, ssm_disc disc,
                                   ssm_dtype compute, int32_t with_backward,
                                   int32_t ckpt_every, const ssm_tuning* tuning) {
  g_last_error.clear();
  if (validate_seqs(seqs, n_seq) != SSM_OK) return 0;
  bool any = false;
  const std::vector<ssm_seq_desc> d = with_caps(seqs, n_seq, &any);
  ssm_plan_s P;
  if (build_plan(P, d.data(), n_seq, disc, compute, with_backward, ckpt_every, tuning, any) != SSM_OK)
    return 0;
  if (!any) return P.ws_bytes;
  // automatic N: the plan of the chosen N must fit as well. Its layout
  // depends on N through the launch mode (sequences ending at different
  // stages launch persistently) and the fused passes, so take the largest
  // over every uniform step down from the caps, in both launch modes unless
  // the tuning fixes one.
  size_t most = P.ws_bytes;
  int maxcap = 0;
  for (const ssm_seq_desc& x : d) maxcap = std::max(maxcap, x.N);
  ssm_tuning tn{};
  if (tuning) tn = *tuning;
  for (int delta = 0; delta <= maxcap; ++delta) {
    std::vector<ssm_seq_desc> dd(seqs, seqs + n_seq);
    for (int i = 0; i < n_seq; ++i)
      if (seqs[i].N < 0) dd[i].N = std::max(0, d[i].N - delta);
    for (int mode : {SSM_LAUNCH_PER_STAGE, SSM_LAUNCH_PERSISTENT}) {
      if (tn.launch != SSM_LAUNCH_AUTO && tn.launch != mode) continue;
      if (mode == SSM_LAUNCH_PERSISTENT && tn.final_state) continue;
      ssm_tuning t2 = tn;
      t2.launch = mode;
      ssm_plan_s Q;
      if (build_plan(Q, dd.data(), n_seq, disc, compute, with_backward, ckpt_every, &t2) == SSM_OK)
        most = std::max(most, Q.ws_bytes);
    }
  }
  g_last_error.clear();
  return most;
}

}  // extern "C"

// the precomputation for descriptors whose N are all resolved
static ssm_status prepare_impl(const ssm_seq_desc* seqs, int32_t n_seq, const ssm_params* sets,
                               int32_t n_sets, ssm_disc disc, ssm_dtype compute,
                               int32_t with_backward, int32_t ckpt_every,
                               const ssm_tuning* tuning, void* ws, size_t ws_bytes,
                               hipStream_t stream, bool norms_region, ssm_plan* out);

extern "C" {

ssm_status ssm_cascade_prepare(const ssm_seq_desc* seqs, int32_t n_seq, const ssm_params* sets,
                               int32_t n_sets, ssm_disc disc, ssm_dtype compute,
                               int32_t with_backward, int32_t ckpt_every,
                               const ssm_tuning* tuning, void* ws, size_t ws_bytes,
                               hipStream_t stream, ssm_plan* out) {
  g_last_error.clear();
  if (!out) return fail(SSM_E_INVALID, "out is NULL");
  *out = nullptr;
  ssm_status st = validate_seqs(seqs, n_seq);
  if (st != SSM_OK) return st;
  bool any = false;
  const std::vector<ssm_seq_desc> d1 = with_caps(seqs, n_seq, &any);
  if (!any)
    return prepare_impl(seqs, n_seq, sets, n_sets, disc, compute, with_backward, ckpt_every, tuning, ws, ws_bytes,
                        stream, false, out);
  // automatic N: the powers up to each sequence's cap, their Frobenius norms
  // read back (one more synchronization), then the plan with the chosen N
  ssm_plan p1 = nullptr;
  st = prepare_impl(d1.data(), n_seq, sets, n_sets, disc, compute, with_backward, ckpt_every, tuning, ws, ws_bytes,
                    stream, true, &p1);
  if (st != SSM_OK) return st;
  std::vector<double> nrm((size_t)p1->n_norms);
  std::vector<int64_t> base(p1->ops.size(), 0);
  {
    int64_t off = 0;
    for (size_t i = 0; i < p1->ops.size(); ++i) {
      base[i] = off;
      off += p1->ops[i].N + 1;
    }
    unsigned char* meta = p1->ws + p1->r_meta.off;
    hipError_t e = launch_power_norms(reinterpret_cast<const OpDev*>(meta + p1->m_ops), (int)p1->ops.size(),
                                      p1->max_N, p1->at<double>(p1->r_pw), p1->at<double>(p1->r_norms), stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(nrm.data(), p1->ws + p1->r_norms.off, nrm.size() * sizeof(double), hipMemcpyDeviceToHost,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      ssm_cascade_destroy(p1);
      return hip_fail(e, "norms of the powers");
    }
  }
  // N: the smallest n with |Abar^(2^(n+1))|_F <= 10^N given, else the cap
  std::vector<ssm_seq_desc> d2(seqs, seqs + n_seq);
  for (int i = 0; i < n_seq; ++i) {
    if (seqs[i].N >= 0) continue;
    const int op = p1->seqs[i].op;
    const double tol = std::pow(10.0, (double)seqs[i].N);
    int n = d1[i].N;
    for (int c = 0; c < d1[i].N; ++c)
      if (nrm[(size_t)(base[op] + c + 1)] <= tol) {
        n = c;
        break;
      }
    d2[i].N = n;
  }
  ssm_cascade_destroy(p1);
  return prepare_impl(d2.data(), n_seq, sets, n_sets, disc, compute, with_backward, ckpt_every, tuning, ws, ws_bytes,
                      stream, false, out);
}

}  // extern "C"

static ssm_status prepare_impl(const ssm_seq_desc* seqs, int32_t n_seq, const ssm_params* sets,
                               int32_t n_sets, ssm_disc disc, ssm_dtype compute,
                               int32_t with_backward, int32_t ckpt_every,
                               const ssm_tuning* tuning, void* ws, size_t ws_bytes,
                               hipStream_t stream, bool norms_region, ssm_plan* out) {
  if (!out) return fail(SSM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!sets) return fail(SSM_E_INVALID, "sets is NULL");
  if (!ws) return fail(SSM_E_INVALID, "workspace is NULL");
  ssm_plan_s* P = new (std::nothrow) ssm_plan_s();
  if (!P) return fail(SSM_E_INVALID, "out of host memory");
  ssm_status st = build_plan(*P, seqs, n_seq, disc, compute, with_backward, ckpt_every, tuning, norms_region);
  if (st != SSM_OK) {
    delete P;
    return st;
  }
  if (P->n_sets > n_sets) {
    delete P;
    return fail(SSM_E_INVALID, "a sequence uses param_set %d but n_sets is %d", P->n_sets - 1,
                n_sets);
  }
  for (const OpDev& o : P->ops) {
    const ssm_params& ps = sets[o.set];
    if (!ps.A || !ps.B || !ps.C || !ps.D) {
      delete P;
      return fail(SSM_E_INVALID, "parameter set %d has a NULL matrix", o.set);
    }
    if (ps.m != o.m || ps.p != o.p || ps.q != o.q || ps.reserved != 0) {
      delete P;
      return fail(SSM_E_INVALID, "parameter set %d sizes (%d,%d,%d) differ from its sequences",
                  o.set, ps.m, ps.p, ps.q);
    }
  }
  // layout of the flat gradient buffer: every parameter set, in order
  {
    size_t off = 0;
    std::vector<size_t> set_out(n_sets, 0);
    for (int st = 0; st < n_sets; ++st) {
      const ssm_params& ps = sets[st];
      if (ps.m < 0 || ps.p < 0 || ps.q < 0) {
        delete P;
        return fail(SSM_E_INVALID, "parameter set %d has negative sizes", st);
      }
      set_out[st] = off;
      off += (size_t)ps.m * ps.m + (size_t)ps.m * ps.p + (size_t)ps.q * ps.m + (size_t)ps.q * ps.p;
    }
    P->grad_numel = off;
    if (P->with_backward) {
      P->scat.resize(n_sets, ScatterJob{});
      for (int st = 0; st < n_sets; ++st) {
        ScatterJob& j = P->scat[st];
        if (st >= P->n_sets || j.n_ops == 0) {
          j = ScatterJob{};
          j.op_first = 0;
          j.n_ops = 0;
          j.m = sets[st].m;
          j.mp = j.m ? std::max(pad_m(j.m), P->min_mp) : 0;
          j.p = sets[st].p;
          j.q = sets[st].q;
          j.dC = -1;
          j.dD = -1;
        }
        j.out = (int64_t)set_out[st];
      }
    }
  }
  if (ws_bytes < P->ws_bytes) {
    size_t need = P->ws_bytes;
    delete P;
    return fail(SSM_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  if (((uintptr_t)ws) % ALIGN != 0) {
    delete P;
    return fail(SSM_E_INVALID, "workspace must be 256-byte aligned");
  }
  P->ws = static_cast<unsigned char*>(ws);
  P->src.resize(P->ops.size());
  for (size_t i = 0; i < P->ops.size(); ++i) {
    const ssm_params& ps = sets[P->ops[i].set];
    P->src[i] = OpSrc{ps.A, ps.B, ps.C, ps.D};
  }

  // GEMM jobs of the precomputation
  double* pw = P->at<double>(P->r_pw);
  double* bbar = P->at<double>(P->r_bbar);
  double* minv = P->at<double>(P->r_minv);
  double* nmat = P->at<double>(P->r_nmat);
  double* bsc = P->at<double>(P->r_bsc);
  std::vector<GemmJob>& J = P->jobs;
  P->job_kind.clear();
  if (disc == SSM_DISC_TRAPEZOID) {
    // triangular inverse: per level, Y X^-1 into the scratch right half of
    // aug, then -Z^-1 (Y X^-1) into the block of minv (kind 2 groups, gated
    // on the operator's triangular flag)
    double* augp = P->at<double>(P->r_aug);
    const int32_t* tri_d = reinterpret_cast<const int32_t*>(P->ws + P->r_meta.off + P->m_tri);
    for (int sz = 32; sz < P->max_mp; sz *= 2) {
      for (int half = 0; half < 2; ++half) {
        int start = (int)J.size();
        for (size_t oi = 0; oi < P->ops.size(); ++oi) {
          const OpDev& o = P->ops[oi];
          const int mp = o.mp, W = 2 * mp;
          for (int r0 = 0; r0 + 2 * sz <= mp && sz < mp; r0 += 2 * sz) {
            double* Y = augp + o.sc_aug + (int64_t)(r0 + sz) * W + r0;
            double* T = augp + o.sc_aug + (int64_t)(r0 + sz) * W + mp + r0;
            const double* Xi = minv + o.minv + (int64_t)r0 * mp + r0;
            const double* Zi = minv + o.minv + (int64_t)(r0 + sz) * mp + (r0 + sz);
            double* out = minv + o.minv + (int64_t)(r0 + sz) * mp + r0;
            GemmJob jb = half == 0 ? GemmJob{Y, Xi, T, sz, sz, sz, W, mp, W, 0, 0, 1.0, 0.0}
                                   : GemmJob{Zi, T, out, sz, sz, sz, mp, W, mp, 0, 0, -1.0, 0.0};
            jb.gate = tri_d + oi;
            J.push_back(jb);
          }
        }
        P->job_groups.push_back({start, (int)J.size() - start});
        P->job_dims.push_back({sz, sz});
        P->job_kind.push_back(2);
      }
    }
    int start = (int)J.size(), mx = 0, mxn = 0;
    for (const OpDev& o : P->ops) {
      // Abar = M^{-1} (I + h A)
      J.push_back(GemmJob{minv + o.minv, nmat + o.sc_n, pw + o.pw, o.mp, o.mp, o.mp, o.mp, o.mp,
                          o.mp, 0, 0, 1.0, 0.0});
      // Bbar = M^{-1} (delta B)
      J.push_back(GemmJob{minv + o.minv, bsc + o.sc_b, bbar + o.bbar, o.mp, o.p, o.mp, o.mp, o.p,
                          o.p, 0, 0, 1.0, 0.0});
      mx = std::max(mx, o.mp);
      mxn = std::max(mxn, o.mp);
    }
    P->job_groups.push_back({start, (int)J.size() - start});
    P->job_dims.push_back({mx, mxn});
    P->job_kind.push_back(0);
  }
  // the lower-triangular mark of operator i (set on the device before the
  // squarings): where it is set, every power is lower triangular and the
  // products with a power below leave out the zero K ranges
  const OpDev* ops_dev = reinterpret_cast<const OpDev*>(P->ws + P->r_meta.off + P->m_ops);
  auto low = [&](const OpDev& o) { return &ops_dev[&o - P->ops.data()].lower; };
  for (int kk = 0; kk < P->max_N; ++kk) {  // P_{k+1} = P_k P_k
    int start = (int)J.size(), mx = 0;
    for (const OpDev& o : P->ops) {
      if (o.N <= kk) continue;
      const int64_t mm = (int64_t)o.mp * o.mp;
      double* Pk = pw + o.pw + kk * mm;
      J.push_back(GemmJob{Pk, Pk, Pk + mm, o.mp, o.mp, o.mp, o.mp, o.mp, o.mp, 0, 0, 1.0, 0.0, nullptr, low(o), 1 | 4});
      mx = std::max(mx, o.mp);
    }
    P->job_groups.push_back({start, (int)J.size() - start});
    P->job_dims.push_back({mx, mx});
    P->job_kind.push_back(0);
  }
  // K_j = [Bbar, Abar Bbar, ...] by doubling: K_0 = Bbar; K_{i+1} = [K_i | P_i K_i]
  if (P->max_kry > 0) {
    double* kw = P->at<double>(P->r_kw);
    int start = (int)J.size(), mx = 0, mn = 0;
    for (const OpDev& o : P->ops) {
      if (o.kry <= 0) continue;
      J.push_back(GemmJob{bbar + o.bbar, nullptr, kw + o.kw, o.mp, o.p, 0, o.p, 0, o.kst, 0, 0, 1.0,
                          0.0});
      mx = std::max(mx, o.mp);
      mn = std::max(mn, o.p);
    }
    P->job_groups.push_back({start, (int)J.size() - start});
    P->job_dims.push_back({mx, mn});
    P->job_kind.push_back(1);
    for (int i = 0; i < P->max_kry; ++i) {
      start = (int)J.size();
      mx = mn = 0;
      for (const OpDev& o : P->ops) {
        if (o.kry <= i) continue;
        const int64_t mm = (int64_t)o.mp * o.mp;
        const int w = o.p << i;
        J.push_back(GemmJob{pw + o.pw + i * mm, kw + o.kw, kw + o.kw + w, o.mp, w, o.mp, o.mp, o.kst,
                            o.kst, 0, 0, 1.0, 0.0, nullptr, low(o), 1});
        mx = std::max(mx, o.mp);
        mn = std::max(mn, w);
      }
      if ((int)J.size() > start) {
        P->job_groups.push_back({start, (int)J.size() - start});
        P->job_dims.push_back({mx, mn});
        P->job_kind.push_back(0);
      }
    }
  }

  // C P_l for the tail pairs: C (q x m, the caller's FP64 matrix) times the
  // power of the last stage
  bool any_cp = false;
  {
    double* kw = P->at<double>(P->r_kw);
    int start = (int)J.size(), mx = 0, mn = 0;
    for (int i = 0; i < P->n_ops; ++i) {
      const OpDev& o = P->ops[i];
      if (o.cpl < 0) continue;
      const int64_t mm = (int64_t)o.mp * o.mp;
      J.push_back(GemmJob{P->src[i].C, pw + o.pw + o.cpl * mm, kw + o.cpw, o.q, o.mp, o.m, o.m, o.mp,
                          o.mp, 0, 0, 1.0, 0.0, nullptr, low(o), 4});
      mx = std::max(mx, o.q);
      mn = std::max(mn, o.mp);
    }
    if ((int)J.size() > start) {
      P->job_groups.push_back({start, (int)J.size() - start});
      P->job_dims.push_back({mx, mn});
      P->job_kind.push_back(0);
      any_cp = true;
    }
  }

  // G_j = C Abar^(j 2^k0), j < 2^s, for the output folds: G_0 = C, then by
  // doubling, [G_{2^t} .. G_{2^{t+1}-1}] = [G_0 .. G_{2^t - 1}] P_{k0+t}
  bool any_fold = false;
  {
    double* kw = P->at<double>(P->r_kw);
    int start = (int)J.size(), mx = 0, mn = 0;
    for (int i = 0; i < P->n_ops; ++i) {
      const OpDev& o = P->ops[i];
      if (o.fold_s <= 0) continue;
      J.push_back(GemmJob{P->src[i].C, nullptr, kw + o.fold_gw, o.q, o.m, 0, o.m, 0, o.mp, 0, 0, 1.0, 0.0});
      mx = std::max(mx, o.q);
      mn = std::max(mn, o.m);
    }
    if ((int)J.size() > start) {
      P->job_groups.push_back({start, (int)J.size() - start});
      P->job_dims.push_back({mx, mn});
      P->job_kind.push_back(1);
      any_fold = true;
    }
    // G_{2^t .. 2^(t+1) - 1} = G_{0 .. 2^t - 1} P_{k0 + t}, one doubling per
    // folded stage (up to six)
    int max_fold = 0;
    for (const OpDev& o : P->ops) max_fold = std::max(max_fold, (int)o.fold_s);
    for (int t = 0; t < max_fold; ++t) {
      start = (int)J.size();
      mx = mn = 0;
      for (const OpDev& o : P->ops) {
        if (o.fold_s <= t) continue;
        const int64_t mm = (int64_t)o.mp * o.mp;
        const int rows = 16 << t;
        J.push_back(GemmJob{kw + o.fold_gw, pw + o.pw + (o.fold_k0 + t) * mm, kw + o.fold_gw + (int64_t)rows * o.mp,
                            rows, o.mp, o.mp, o.mp, o.mp, o.mp, 0, 0, 1.0, 0.0, nullptr, low(o), 4});
        mx = std::max(mx, rows);
        mn = std::max(mn, o.mp);
      }
      if ((int)J.size() > start) {
        P->job_groups.push_back({start, (int)J.size() - start});
        P->job_dims.push_back({mx, mn});
        P->job_kind.push_back(0);
      }
    }
  }

  // host image of the meta region
  P->meta_host.assign(P->meta_bytes, 0);
  std::memcpy(P->meta_host.data() + P->m_seqs, P->seqs.data(), sizeof(SeqDev) * P->seqs.size());
  std::memcpy(P->meta_host.data() + P->m_ops, P->ops.data(), sizeof(OpDev) * P->ops.size());
  std::memcpy(P->meta_host.data() + P->m_src, P->src.data(), sizeof(OpSrc) * P->src.size());
  if (!P->tiles.empty())
    std::memcpy(P->meta_host.data() + P->m_tiles, P->tiles.data(),
                sizeof(Tile) * P->tiles.size());
  if (!J.empty())
    std::memcpy(P->meta_host.data() + P->m_jobs, J.data(), sizeof(GemmJob) * J.size());
  if (!P->ranges.empty())
    std::memcpy(P->meta_host.data() + P->m_ranges, P->ranges.data(),
                sizeof(ResRange) * P->ranges.size());
  if (!P->chain_units.empty())
    std::memcpy(P->meta_host.data() + P->m_chain, P->chain_units.data(),
                sizeof(ChainUnit) * P->chain_units.size());
  if (!P->pair_units.empty())
    std::memcpy(P->meta_host.data() + P->m_pair, P->pair_units.data(),
                sizeof(PairUnit) * P->pair_units.size());
  if (!P->input_units.empty())
    std::memcpy(P->meta_host.data() + P->m_input, P->input_units.data(),
                sizeof(ResRange) * P->input_units.size());
  if (!P->fold_units.empty())
    std::memcpy(P->meta_host.data() + P->m_fold, P->fold_units.data(),
                sizeof(FoldUnit) * P->fold_units.size());
  if (!P->plr_jobs.empty()) {
    unsigned char* mh = P->meta_host.data();
    std::memcpy(mh + P->m_plr_jobs, P->plr_jobs.data(), sizeof(PlrJob) * P->plr_jobs.size());
    std::memcpy(mh + P->m_plr_recoff, P->plr_rec_off.data(), sizeof(int64_t) * P->plr_rec_off.size());
    std::memcpy(mh + P->m_plr_rankoff, P->plr_rank_off.data(), sizeof(int32_t) * P->plr_rank_off.size());
    if (!P->plr_units.empty())
      std::memcpy(mh + P->m_plr_units, P->plr_units.data(), sizeof(PlrUnit) * P->plr_units.size());
  }
  if (P->launch == SSM_LAUNCH_PERSISTENT) {
    unsigned char* mh = P->meta_host.data();
    if (!P->items.empty())
      std::memcpy(mh + P->m_items, P->items.data(), sizeof(PItem) * P->items.size());
    if (!P->ritems.empty())
      std::memcpy(mh + P->m_ritems, P->ritems.data(), sizeof(RItem) * P->ritems.size());
    if (!P->cnt_target.empty())
      std::memcpy(mh + P->m_cnttarget, P->cnt_target.data(), sizeof(int32_t) * P->cnt_target.size());
    std::memcpy(mh + P->m_cntoff, P->cnt_off.data(), sizeof(int32_t) * P->cnt_off.size());
    std::memcpy(mh + P->m_ntiles, P->ntiles.data(), sizeof(int32_t) * P->ntiles.size());
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
      ncu = 256;
    if (P->persist_res) {  // one workgroup of 8 waves per compute unit (LDS and registers)
      P->persistent_grid = (int)std::min<int64_t>(ncu, (int64_t)P->ritems.size());
    } else {
      const int64_t g = (int64_t)persistent_blocks_per_cu(P->compute) * ncu;
      P->persistent_grid = (int)std::min<int64_t>(g, (int64_t)P->items.size());
    }
  }
  if (P->with_backward) {
    plan_backward_jobs(*P);
    unsigned char* mh = P->meta_host.data();
    if (!P->chunks.empty())
      std::memcpy(mh + P->m_chunks, P->chunks.data(), sizeof(RedChunk) * P->chunks.size());
    size_t o = P->m_sj;
    for (auto* v : {&P->sj_dp, &P->sj_dbb, &P->sj_dc, &P->sj_dd}) {
      if (!v->empty()) std::memcpy(mh + o, v->data(), sizeof(SumJob) * v->size());
      o += sizeof(SumJob) * v->size();
    }
    if (!P->set_ops.empty())
      std::memcpy(mh + P->m_set_ops, P->set_ops.data(), sizeof(int32_t) * P->set_ops.size());
    if (P->m_scat + sizeof(ScatterJob) * P->scat.size() > P->m_bjobs) {
      delete P;
      return fail(SSM_E_INVALID, "too many parameter sets for the plan tables");
    }
    if (!P->scat.empty())
      std::memcpy(mh + P->m_scat, P->scat.data(), sizeof(ScatterJob) * P->scat.size());
    if (!P->bjobs.empty())
      std::memcpy(mh + P->m_bjobs, P->bjobs.data(), sizeof(GemmJob) * P->bjobs.size());
  }

  unsigned char* meta = P->ws + P->r_meta.off;
  const OpDev* ops_d = reinterpret_cast<const OpDev*>(meta + P->m_ops);
  const OpSrc* src_d = reinterpret_cast<const OpSrc*>(meta + P->m_src);
  int* status_d = reinterpret_cast<int*>(meta + P->m_status);
  const GemmJob* jobs_d = reinterpret_cast<const GemmJob*>(meta + P->m_jobs);

  auto bail = [&](ssm_status s) {
    delete P;
    return s;
  };
  hipError_t e = hipMemcpyAsync(meta, P->meta_host.data(), P->meta_bytes, hipMemcpyHostToDevice,
                                stream);
  if (e != hipSuccess) return bail(hip_fail(e, "upload of plan tables"));
  const int given = disc == SSM_DISC_GIVEN;
  if (P->r_kw.bytes > 0) {
    e = launch_zero_i32(P->at<int32_t>(P->r_kw), (int64_t)(P->r_kw.bytes / 4), stream);
    if (e != hipSuccess) return bail(hip_fail(e, "zero fill"));
  }
  size_t g = 0;
  if (disc == SSM_DISC_ZOH) {
    const ssm_status zs = zoh_discretize(*P, ops_d, src_d, stream);
    if (zs != SSM_OK) return bail(zs);
  } else {
    e = launch_disc_setup(ops_d, P->n_ops, src_d, given, P->at<double>(P->r_aug), nmat, bsc, pw,
                          bbar, P->max_mp, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "discretization setup launch"));
  }
  if (disc == SSM_DISC_TRAPEZOID) {
    // M^{-1}: blockwise for lower-triangular M, Gauss-Jordan otherwise
    int32_t* tri_d = reinterpret_cast<int32_t*>(meta + P->m_tri);
    double* tscale_d = reinterpret_cast<double*>(meta + P->m_tri_scale);
    e = launch_tri_check(ops_d, P->n_ops, src_d, tri_d, tscale_d, stream);
    if (e == hipSuccess)
      e = launch_tri_diag_inv(ops_d, P->n_ops, P->max_mp, P->at<double>(P->r_aug), minv, tri_d, tscale_d, status_d,
                              stream);
    if (e != hipSuccess) return bail(hip_fail(e, "triangular inverse launch"));
    for (; g < P->job_groups.size() && P->job_kind[g] == 2; ++g) {
      const auto& grp = P->job_groups[g];
      e = launch_gemm_f64(jobs_d + grp.first, grp.second, P->job_dims[g].first, P->job_dims[g].second, stream);
      if (e != hipSuccess) return bail(hip_fail(e, "triangular inverse GEMM launch"));
    }
    e = launch_gauss_jordan(ops_d, P->n_ops, P->at<double>(P->r_aug), minv, status_d, tri_d, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "Gauss-Jordan launch"));
    const auto& grp = P->job_groups[g];
    e = launch_gemm_f64(jobs_d + grp.first, grp.second, P->job_dims[g].first,
                        P->job_dims[g].second, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "discretization GEMM launch"));
    ++g;
  }
  // Abar (P_0) is complete: mark the operators whose Abar is lower triangular
  e = launch_mark_lower(reinterpret_cast<OpDev*>(meta + P->m_ops), P->n_ops, pw, stream);
  if (e != hipSuccess) return bail(hip_fail(e, "triangular mark launch"));
  for (; g < P->job_groups.size(); ++g) {
    const auto& grp = P->job_groups[g];
    if (P->job_kind[g] == 1)
      e = launch_axpy(jobs_d + grp.first, grp.second, P->job_dims[g].first, P->job_dims[g].second,
                      stream);
    else
      e = launch_gemm_f64(jobs_d + grp.first, grp.second, P->job_dims[g].first,
                          P->job_dims[g].second, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "squaring GEMM launch"));
  }
  if (P->max_kry > 0 || any_cp) {
    e = launch_pack_krylov(ops_d, P->n_ops, P->at<double>(P->r_kw), P->ws + P->r_pc.off, P->compute,
                           P->max_mp, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "Krylov pack launch"));
  }
  if (any_fold) {
    e = launch_pack_fold(ops_d, P->n_ops, P->at<double>(P->r_kw), P->ws + P->r_pc.off, P->compute, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "fold pack launch"));
  }
  e = launch_pack(ops_d, P->n_ops, src_d, pw, bbar, P->ws + P->r_pc.off, P->compute,
                  P->with_backward, P->ws + P->r_small.off, P->state_f64, P->max_mp, P->max_N,
                  stream);
  if (e != hipSuccess) return bail(hip_fail(e, "pack launch"));
  if (!P->plr_jobs.empty()) {
    // PLR forms of the eligible stages' powers, and their ranks read back
    PlrCompressParams cp{};
    cp.ops = ops_d;
    cp.jobs = reinterpret_cast<const PlrJob*>(meta + P->m_plr_jobs);
    cp.pw = pw;
    cp.rec = P->ws + P->r_plr.off;
    cp.rec_off = reinterpret_cast<const int64_t*>(meta + P->m_plr_recoff);
    cp.ranks = P->at<int32_t>(P->r_plr_rank);
    cp.rank_off = reinterpret_cast<const int32_t*>(meta + P->m_plr_rankoff);
    cp.qs = P->at<double>(P->r_plr_q);
    const double tol = std::pow(10.0, -(double)P->plr_digits);
    cp.tol2 = tol * tol;
    e = launch_zero_i32(cp.ranks, (int64_t)(P->r_plr_rank.bytes / 4), stream);
    if (e == hipSuccess) e = launch_plr_compress(P->compute, cp, (int)P->plr_jobs.size(), P->plr_max_s, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "PLR compression launch"));
    e = hipMemcpyAsync(P->plr_ranks_host.data(), cp.ranks, P->r_plr_rank.bytes, hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "PLR rank read"));
  }
  int status_h[4] = {0, 0, 0, 0};
  e = hipMemcpyAsync(status_h, status_d, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return bail(hip_fail(e, "status read"));
  // the operator table as the device left it (the lower-triangular marks)
  std::vector<OpDev> ops_back(P->ops.size());
  e = hipMemcpyAsync(ops_back.data(), ops_d, sizeof(OpDev) * ops_back.size(), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return bail(hip_fail(e, "operator table read"));
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bail(hip_fail(e, "prepare synchronization"));
  if (status_h[0] != 0)
    return bail(fail(SSM_E_NUMERIC, "I - delta/2 A is singular to working precision"));
  for (size_t i = 0; i < P->ops.size(); ++i) P->ops[i].lower = ops_back[i].lower;
  for (int c = 0; c < 4; ++c) {
    P->class_lower[c] = 1;
    for (const OpDev& o : P->ops)
      if (o.mp == kClassMp[c] && !o.lower) P->class_lower[c] = 0;
  }
  if (!P->plr_jobs.empty()) plr_select(*P);
  *out = P;
  return SSM_OK;
}

extern "C" {

// the forward apply; x0 (nullable) is x_{-1} of every sequence, packed in
// sequence order, m of each, in the plan's state type
// xb0, xb1: the two state buffers (the plan's own, or the static scratch of
// ssm_cascade_apply_noalloc); timed: record timing events if timing is on
static ssm_status apply_impl(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel, const void* x0,
                             size_t x0_numel, void* y, size_t y_numel, hipStream_t stream,
                             unsigned char* xb0, unsigned char* xb1, bool timed, void* x_last = nullptr,
                             size_t x_last_numel = 0) {
  ssm_plan_s& P = *plan;
  ssm_status st = check_io(P, u, u_dtype, u_numel, y, y_numel, "y");
  if (st != SSM_OK) return st;
  size_t want_state = 0;
  for (int i = 0; i < P.n_seq; ++i) want_state += (size_t)P.ops[P.seqs[i].op].m;
  if (x_last) {
    if (!P.final_state)
      return fail(SSM_E_NOT_PREPARED, "x_last needs a plan prepared with ssm_tuning.final_state = 1");
    if (x_last_numel != want_state)
      return fail(SSM_E_INVALID, "x_last_numel %zu, the sequences' states need %zu", x_last_numel, want_state);
  }
  if (x0) {
    const size_t want = want_state;
    if (x0_numel != want)
      return fail(SSM_E_INVALID, "x0_numel %zu, the sequences' states need %zu", x0_numel, want);
    if (P.launch == SSM_LAUNCH_PERSISTENT)
      return fail(SSM_E_UNSUPPORTED, "an initial state needs per-stage launches (the plan is persistent)");
    if (P.state_bf16)
      return fail(SSM_E_UNSUPPORTED, "an initial state needs an FP32 or FP64 state (the plan keeps BF16)");
  }
  if (P.launch == SSM_LAUNCH_PERSISTENT && P.persist_res) {
    unsigned char* meta = P.ws + P.r_meta.off;
    RPersistParams pp{};
    pp.base = base_params(P, 0);
    pp.base.tiles = nullptr;
    pp.base.src = u;
    pp.base.src_dtype = (int)u_dtype;
    pp.base.dst = y;
    pp.base.flags = SF_EPILOGUE;
    pp.items = reinterpret_cast<const RItem*>(meta + P.m_ritems);
    pp.n_items = (int32_t)P.ritems.size();
    pp.counters = reinterpret_cast<int32_t*>(meta + P.m_counters);
    pp.cnt_off = reinterpret_cast<const int32_t*>(meta + P.m_cntoff);
    pp.cnt_target = reinterpret_cast<const int32_t*>(meta + P.m_cnttarget);
    pp.x0 = xb0;
    pp.x1 = xb1;
    pp.flag = pp.counters + P.n_counters;
    pp.spin_limit = P.spin_limit;
    hipError_t e = launch_zero_i32(pp.counters, P.n_counters + 1, stream);
    if (e != hipSuccess) return hip_fail(e, "counter reset launch");
    TimedLaunch tl(P, stream, 0, timed);
    e = launch_persist_res(P.compute, pp, P.persistent_grid, P.persist_lds, stream);
    if (e != hipSuccess) return hip_fail(e, "persistent launch");
    tl.done();
    return SSM_OK;
  }
  if (P.launch == SSM_LAUNCH_PERSISTENT) {
    unsigned char* meta = P.ws + P.r_meta.off;
    PersistParams pp{};
    pp.base = base_params(P, 0);
    pp.base.tiles = nullptr;
    pp.base.src = u;
    pp.base.src_dtype = (int)u_dtype;
    pp.base.dst = y;
    pp.base.flags = SF_EPILOGUE;
    pp.items = reinterpret_cast<const PItem*>(meta + P.m_items);
    pp.n_items = (int32_t)P.items.size();
    pp.counters = reinterpret_cast<int32_t*>(meta + P.m_counters);
    pp.cnt_off = reinterpret_cast<const int32_t*>(meta + P.m_cntoff);
    pp.ntiles = reinterpret_cast<const int32_t*>(meta + P.m_ntiles);
    pp.x0 = xb0;
    pp.x1 = xb1;
    pp.flag = pp.counters + P.n_counters;
    pp.spin_limit = P.spin_limit;
    hipError_t e = launch_zero_i32(pp.counters, P.n_counters + 1, stream);
    if (e != hipSuccess) return hip_fail(e, "counter reset launch");
    TimedLaunch tl(P, stream, 0, timed);
    e = launch_persistent(P.compute, pp, P.persistent_grid, stream);
    if (e != hipSuccess) return hip_fail(e, "persistent launch");
    tl.done();
    return SSM_OK;
  }
  for (int c = 0; c < 4; ++c) {
    if (P.class_tile_count[c] == 0) continue;
    StageParams prm = base_params(P, c);
    prm.src = u;
    prm.src_dtype = (int)u_dtype;
    prm.dst = y;
    prm.adjoint = 0;
    hipError_t e = hipSuccess;
    if (!P.class_all_kry[c]) {
      // V^(0) = Bbar U into the first state buffer
      prm.xout = xb0;
      prm.n_tiles = P.class_tile_count[c];
      e = launch_project(kClassMp[c], P.state_f64, P.class_bm[c], prm, stream);
      if (e != hipSuccess) return hip_fail(e, "projection launch");
    }
    // (final_state: every epilogue also stores the state rows it finishes)
    prm.flags = SF_EPILOGUE | (P.final_state ? SF_STORE_AT_EPI : 0);
    int k_begin = 0;
    if (P.max_kry > 0 && res_supported(kClassMp[c], P.compute)) {
      // the leading stages folded into the input pass, x^(kry) in buffer kry % 2
      prm.xin = xb0;
      prm.xout = xb1;
      if (P.class_input_count[c] > 0) {
        const ResRange* un = reinterpret_cast<const ResRange*>(P.ws + P.r_meta.off + P.m_input) +
                             P.class_input_start[c];
        e = launch_input_split(kClassMp[c], P.compute, P.class_input_p[c], P.class_input_kdim[c],
                               P.state_bf16 != 0, prm, un, P.class_input_count[c], P.class_input_lds[c],
                               stream);
      } else {
        const ResRange* rg = reinterpret_cast<const ResRange*>(P.ws + P.r_meta.off + P.m_ranges) +
                             P.class_range_start[c];
        e = launch_krylov_res(kClassMp[c], P.compute, prm, rg, P.class_range_count[c], stream);
      }
      if (e != hipSuccess) return hip_fail(e, "input pass launch");
      prm.skip_kry = 1;
      k_begin = P.class_min_kry[c];
    }
    if (x0) {  // x_{-1}: Abar^(l+1) x0 into the rows the first pass has finished
      unsigned char* meta = P.ws + P.r_meta.off;
      e = launch_inject_x0(kClassMp[c], P.state_f64 != 0, reinterpret_cast<const SeqDev*>(meta + P.m_seqs), P.n_seq,
                           reinterpret_cast<const OpDev*>(meta + P.m_ops), P.at<double>(P.r_pw), x0,
                           xb0, xb1, P.ws + P.r_small.off, y, P.final_state != 0, stream);
      if (e != hipSuccess) return hip_fail(e, "initial state launch");
    }
    if (P.fold_mixed[c]) {
      // ragged class: stage pairs from the input pass on (each sequence up to
      // its own fold), then the folds, each group reading the buffer its
      // sequences' last pair wrote
      int cur = k_begin & 1;
      for (int kk = k_begin; kk < (int)P.pair_count[c].size() && P.pair_count[c][kk] > 0; kk += 2) {
        prm.k = kk;
        prm.xin = (cur ? xb1 : xb0);
        prm.xout = (cur ? xb0 : xb1);
        TimedLaunch tl(P, stream, 4, timed);
        const PairUnit* un = reinterpret_cast<const PairUnit*>(P.ws + P.r_meta.off + P.m_pair) +
                             P.pair_start[c][kk];
        e = launch_stage_pair(kClassMp[c], P.compute, prm, un, P.pair_count[c][kk], false, P.state_bf16 != 0,
                              P.pair_lds_bytes[c][kk], stream);
        if (e != hipSuccess) return hip_fail(e, "stage pair launch");
        tl.done();
        cur ^= 1;
      }
      for (const auto& fl : P.mixed_folds) {
        if (fl.c != c) continue;
        prm.xin = (fl.buf ? xb1 : xb0);
        prm.xout = (fl.buf ? xb0 : xb1);
        TimedLaunch tl(P, stream, 5, timed);
        const FoldUnit* un = reinterpret_cast<const FoldUnit*>(P.ws + P.r_meta.off + P.m_fold) + fl.start;
        e = fl.wide ? launch_output_fold_wide(kClassMp[c], P.compute, P.state_bf16 != 0, fl.max_p, fl.q4, prm, un,
                                              fl.count, stream)
                    : launch_output_fold(kClassMp[c], P.compute, fl.s, P.state_bf16 != 0, prm, un, fl.count,
                                         fl.lds, stream);
        if (e != hipSuccess) return hip_fail(e, "output fold launch");
        tl.done();
      }
      continue;
    }
    // the input of stage kk is in buffer kk % 2 until the first stage pair;
    // from there on every sequence of the class runs every stage, and the
    // buffers simply alternate per launch
    int cur = k_begin & 1;
    for (int kk = k_begin; kk <= P.class_max_last[c];) {
      prm.k = kk;
      prm.xin = (cur ? xb1 : xb0);
      prm.xout = (cur ? xb0 : xb1);
      prm.n_tiles = P.class_active[c][kk];
      if (P.fold_s[c] > 0 && kk == P.fold_k0[c]) {  // the remaining stages and y in one pass
        TimedLaunch tl(P, stream, 5, timed);
        const FoldUnit* un = reinterpret_cast<const FoldUnit*>(P.ws + P.r_meta.off + P.m_fold) + P.fold_start[c];
        e = P.fold_wide[c] ? launch_output_fold_wide(kClassMp[c], P.compute, P.state_bf16 != 0, P.fold_max_p[c], P.fold_q4[c],
                                                     prm, un, P.fold_count[c], stream)
                           : launch_output_fold(kClassMp[c], P.compute, P.fold_s[c], P.state_bf16 != 0, prm, un,
                                                P.fold_count[c], P.fold_lds_bytes[c], stream);
        if (e != hipSuccess) return hip_fail(e, "output fold launch");
        tl.done();
        break;
      }
      if (kk < (int)P.plr_use[c].size() && P.plr_use[c][kk]) {  // P_k in PLR form
        TimedLaunch tl(P, stream, 6, timed);
        unsigned char* meta = P.ws + P.r_meta.off;
        PlrStageParams sp{};
        sp.seqs = prm.seqs;
        sp.units = reinterpret_cast<const PlrUnit*>(meta + P.m_plr_units) + P.plr_start[c];
        sp.n_units = P.plr_count[c];
        sp.k = kk;
        sp.rec = P.ws + P.r_plr.off;
        sp.rec_off = reinterpret_cast<const int64_t*>(meta + P.m_plr_recoff);
        sp.ranks = P.at<int32_t>(P.r_plr_rank);
        sp.rank_off = reinterpret_cast<const int32_t*>(meta + P.m_plr_rankoff);
        sp.xin = prm.xin;
        sp.xout = prm.xout;
        e = launch_stage_plr(kClassMp[c], P.compute, sp, stream);
        if (e != hipSuccess) return hip_fail(e, "PLR stage launch");
        tl.done();
        cur ^= 1;
        ++kk;
        continue;
      }
      const bool pair = kk < (int)P.pair_count[c].size() && P.pair_count[c][kk] > 0;
      TimedLaunch tl(P, stream, pair ? 4 : 0, timed);
      if (pair) {
        const PairUnit* un = reinterpret_cast<const PairUnit*>(P.ws + P.r_meta.off + P.m_pair) +
                             P.pair_start[c][kk];
        e = launch_stage_pair(kClassMp[c], P.compute, prm, un, P.pair_count[c][kk],
                              P.pair_tail[c][kk] != 0, P.state_bf16 != 0, P.pair_lds_bytes[c][kk], stream);
      } else {
        e = launch_stage_any(P, c, prm, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "stage launch");
      tl.done();
      cur ^= 1;
      kk += pair ? 2 : 1;
    }
  }
  if (x_last) {  // row L - 1 of each sequence's final state (buffer (last + 1) mod 2)
    unsigned char* meta = P.ws + P.r_meta.off;
    hipError_t e = launch_gather_last(P.state_f64 != 0, reinterpret_cast<const SeqDev*>(meta + P.m_seqs), P.n_seq,
                                      reinterpret_cast<const OpDev*>(meta + P.m_ops), xb0, xb1, x_last, stream);
    if (e != hipSuccess) return hip_fail(e, "final state launch");
  }
  return SSM_OK;
}

// the plan's own state buffers, or an error for a plan prepared without them
static ssm_status own_state(ssm_plan plan, const char* what) {
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (plan->static_state)
    return fail(SSM_E_NOT_PREPARED,
                "%s: the plan was prepared with static_state (no state buffers in its workspace); "
                "apply it with ssm_cascade_apply_noalloc", what);
  return SSM_OK;
}

ssm_status ssm_cascade_apply(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                             void* y, size_t y_numel, hipStream_t stream) {
  g_last_error.clear();
  ssm_status st = own_state(plan, "ssm_cascade_apply");
  if (st != SSM_OK) return st;
  return apply_impl(plan, u, u_dtype, u_numel, nullptr, 0, y, y_numel, stream, plan->ws + plan->r_x0.off,
                    plan->ws + plan->r_x1.off, true);
}

ssm_status ssm_cascade_apply_x0(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                const void* x0, size_t x0_numel, void* y, size_t y_numel,
                                hipStream_t stream) {
  g_last_error.clear();
  if (!x0) return fail(SSM_E_INVALID, "x0 is NULL (ssm_cascade_apply runs from a zero state)");
  ssm_status st = own_state(plan, "ssm_cascade_apply_x0");
  if (st != SSM_OK) return st;
  return apply_impl(plan, u, u_dtype, u_numel, x0, x0_numel, y, y_numel, stream, plan->ws + plan->r_x0.off,
                    plan->ws + plan->r_x1.off, true);
}

ssm_status ssm_cascade_apply_state(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                   const void* x0, size_t x0_numel, void* y, size_t y_numel, void* x_last,
                                   size_t x_last_numel, hipStream_t stream) {
  g_last_error.clear();
  ssm_status st = own_state(plan, "ssm_cascade_apply_state");
  if (st != SSM_OK) return st;
  return apply_impl(plan, u, u_dtype, u_numel, x0, x0 ? x0_numel : 0, y, y_numel, stream,
                    plan->ws + plan->r_x0.off, plan->ws + plan->r_x1.off, true, x_last, x_last_numel);
}

ssm_status ssm_cascade_apply_noalloc(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                     void* y, size_t y_numel, hipStream_t stream) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  ssm_plan_s& P = *plan;
  const size_t one = align_up(P.x_buf_bytes);
  const size_t cap = static_scratch_bytes();
  if (2 * one > cap)
    return fail(SSM_E_WORKSPACE,
                "ssm_cascade_apply_noalloc: the plan's two state buffers need %zu bytes, the static "
                "scratch holds %zu",
                2 * one, cap);
  void* base = nullptr;
  hipError_t e = static_scratch(&base);
  if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
  unsigned char* b0 = static_cast<unsigned char*>(base);
  return apply_impl(plan, u, u_dtype, u_numel, nullptr, 0, y, y_numel, stream, b0, b0 + one, false);
}

ssm_status ssm_cascade_recursion(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                 size_t u_numel, void* y, size_t y_numel, hipStream_t stream) {
  g_last_error.clear();
  ssm_status st = own_state(plan, "ssm_cascade_recursion");
  if (st != SSM_OK) return st;
  ssm_plan_s& P = *plan;
  st = check_io(P, u, u_dtype, u_numel, y, y_numel, "y");
  if (st != SSM_OK) return st;
  unsigned char* meta = P.ws + P.r_meta.off;
  const SeqDev* seqs_d = reinterpret_cast<const SeqDev*>(meta + P.m_seqs);
  const OpDev* ops_d = reinterpret_cast<const OpDev*>(meta + P.m_ops);
  for (int c = 0; c < 4; ++c) {
    if (P.class_tile_count[c] == 0) continue;
    {
      TimedLaunch tl(P, stream, 3);
      hipError_t e = launch_recursion(kClassMp[c], P.compute, seqs_d, P.n_seq, ops_d,
                                      P.at<double>(P.r_pw), P.at<double>(P.r_bbar), u,
                                      (int)u_dtype, P.ws + P.r_x0.off, stream);
      if (e != hipSuccess) return hip_fail(e, "recursion launch");
      tl.done();
    }
    StageParams prm = base_params(P, c);
    prm.src = u;
    prm.src_dtype = (int)u_dtype;
    prm.dst = y;
    prm.flags = SF_NOUPDATE | SF_EPILOGUE;
    prm.xin = P.ws + P.r_x0.off;
    prm.xout = P.ws + P.r_x1.off;
    prm.n_tiles = P.class_tile_count[c];
    hipError_t e = launch_stage(kClassMp[c], P.compute, P.class_bm[c], prm, stream);
    if (e != hipSuccess) return hip_fail(e, "projection launch");
  }
  return SSM_OK;
}

// the backward; x0 (nullable) is x_{-1} of every sequence and dx0 (nullable)
// receives dL/dx_{-1}, both packed in sequence order, m of each
static ssm_status backward_impl(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel, const void* x0,
                                size_t x0_numel, const void* dy, size_t dy_numel, void* du, void* dx0,
                                size_t dx0_numel, double* grad_params, size_t grad_numel, hipStream_t stream) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  ssm_plan_s& P = *plan;
  if (!P.with_backward)
    return fail(SSM_E_NOT_PREPARED, "plan was prepared without with_backward");
  ssm_status st = check_io(P, u, u_dtype, u_numel, dy, dy_numel, "dy");
  if (st != SSM_OK) return st;
  if (grad_params && grad_numel < P.grad_numel)
    return fail(SSM_E_INVALID, "grad_params has %zu elements, needs %zu", grad_numel,
                P.grad_numel);
  {
    size_t want = 0;
    for (int i = 0; i < P.n_seq; ++i) want += (size_t)P.ops[P.seqs[i].op].m;
    if (x0 && x0_numel != want)
      return fail(SSM_E_INVALID, "x0_numel %zu, the sequences' states need %zu", x0_numel, want);
    if (dx0 && dx0_numel != want)
      return fail(SSM_E_INVALID, "dx0_numel %zu, the sequences' states need %zu", dx0_numel, want);
  }
  unsigned char* meta = P.ws + P.r_meta.off;
  const RedChunk* chunks_d = reinterpret_cast<const RedChunk*>(meta + P.m_chunks);
  const SumJob* sj_d = reinterpret_cast<const SumJob*>(meta + P.m_sj);
  const SumJob* sj_dp = sj_d;
  const SumJob* sj_dbb = sj_dp + P.sj_dp.size();
  const SumJob* sj_dc = sj_dbb + P.sj_dbb.size();
  const SumJob* sj_dd = sj_dc + P.sj_dc.size();
  const GemmJob* bj_d = reinterpret_cast<const GemmJob*>(meta + P.m_bjobs);
  const size_t xb = (size_t)P.sum_x * P.x_elem();
  const int c = P.ckpt_every;
  // location of the input of stage k (k = 0..max_last+1)
  auto loc = [&](int k) -> void* {
    if (k % c == 0) return P.ws + P.r_ckpt.off + (size_t)(k / c) * xb;
    return P.ws + P.r_seg.off + (size_t)(k % c - 1) * xb;
  };
  void* W[2] = {P.ws + P.r_x0.off, P.ws + P.r_x1.off};
  void* xfinal = P.ws + P.r_xfinal.off;
  void* gfirst = P.ws + P.r_gfirst.off;
  double* G = P.at<double>(P.r_g);
  const int sdt = P.state_f64 ? DT_F64 : DT_F32;
  const int TO = P.state_f64 ? 64 : 128;
  auto tiles = [&](int a, int b) { return ((a + TO - 1) / TO) * ((b + TO - 1) / TO); };
  hipError_t e;

  for (int cl = 0; cl < 4; ++cl) {
    if (P.class_tile_count[cl] == 0) continue;
    const int mp = kClassMp[cl];
    const int ml = P.class_max_last[cl];
    StageParams prm = base_params(P, cl);
    prm.src = u;
    prm.src_dtype = (int)u_dtype;
    // ---- forward pass keeping stage-input checkpoints and the final states ----
    prm.adjoint = 0;
    prm.xout = loc(0);
    prm.n_tiles = P.class_tile_count[cl];
    e = launch_project(mp, P.state_f64, P.class_bm[cl], prm, stream);
    if (e != hipSuccess) return hip_fail(e, "projection launch");
    if (x0) {  // x_{-1} as the input Abar x_{-1} at row 0
      e = launch_input_x0(mp, P.state_f64 != 0, prm.seqs, P.n_seq, prm.ops, P.at<double>(P.r_pw), x0, loc(0),
                          stream);
      if (e != hipSuccess) return hip_fail(e, "initial state launch");
    }
    prm.flags = 0;
    // the stage inputs x^(1) .. x^(J) straight from u by the resident input
    // pass (x^(j) = K_j [u_l; ...; u_{l-2^j+1}], K_j the first 2^j p columns
    // of the operator's K): one write of the state each instead of a stage's
    // read and write. J: at most every sequence's folded input stages and its
    // last stage (so that the stages from J on still leave its final state),
    // 2^J p <= mp; none with x_{-1}.
    int J = 0;
    if (!x0 && P.stage_kernel != SSM_STAGE_TILED && res_supported(mp, P.compute) && P.class_range_count[cl] > 0) {
      J = 1 << 30;
      for (const SeqDev& s : P.seqs) {
        if (P.ops[s.op].mp != mp) continue;
        int j = std::min(s.kry, s.last);
        while (j > 0 && (s.p << j) > mp) --j;
        J = std::min(J, j);
      }
      if (J == (1 << 30)) J = 0;
    }
    if (J > 0) {
      const ResRange* rg = reinterpret_cast<const ResRange*>(meta + P.m_ranges) + P.class_range_start[cl];
      for (int k = 1; k <= J; ++k) {
        prm.kry_override = k;
        prm.xout = loc(k);
        TimedLaunch tl(P, stream, 0);
        e = launch_krylov_res(mp, P.compute, prm, rg, P.class_range_count[cl], stream);
        if (e != hipSuccess) return hip_fail(e, "input pass launch");
        tl.done();
      }
      prm.kry_override = 0;
    }
    prm.xfinal = xfinal;
    for (int k = J; k <= ml; ++k) {
      prm.k = k;
      prm.xin = loc(k);
      prm.xout = loc(k + 1);
      prm.n_tiles = P.class_active[cl][k];
      TimedLaunch tl(P, stream, 0);
      e = launch_stage_any(P, cl, prm, stream);
      if (e != hipSuccess) return hip_fail(e, "stage launch");
      tl.done();
    }
    prm.xfinal = nullptr;
    // ---- g = C^T dy at every sequence's last stage ----
    prm.adjoint = 1;
    prm.src = dy;
    prm.src_dtype = sdt;
    prm.xout = gfirst;
    prm.n_tiles = P.class_tile_count[cl];
    e = launch_project(mp, P.state_f64, P.class_bm[cl], prm, stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint projection launch");

    RedParams rp{};
    rp.chunks = chunks_d + P.class_chunk_start[cl];
    rp.n_chunks = P.class_chunk_count[cl];
    rp.seqs = prm.seqs;
    rp.u = u;
    rp.dy = dy;
    rp.u_dtype = (int)u_dtype;
    rp.partial = P.ws + P.r_part.off + (size_t)P.class_part_off[cl] * P.x_elem();
    rp.slot_stride = (int64_t)mp * mp;
    const int ncs = P.class_set_count[cl], nco = P.class_op_count[cl];
    const int qm = P.class_max_q[cl], pm = P.class_max_p[cl];
    auto reduce = [&](int a_kind, const void* a_base, const void* a_first, int b_kind,
                      const void* b_base, int k, int ty) -> hipError_t {
      rp.a_kind = a_kind;
      rp.a_base = a_base;
      rp.a_first = a_first;
      rp.b_kind = b_kind;
      rp.b_base = b_base;
      rp.k = k;
      rp.check_last = k >= 0;
      TimedLaunch tl(P, stream, 2);
      // state by state (dL/dP_k) with FP32 state: on the BF16 matrix cores
      // where the stages themselves contract in BF16 (padded m 128, 256),
      // else the FP32 direct-load kernel
      const bool ss = a_kind == RS_STATE && b_kind == RS_STATE && !P.state_f64 && mp >= 64;
      const bool sb = ss && P.compute == DT_BF16 && mp >= 128;
      // one side dy (width q) or u (width p) of at most 16: the thin kernel
      const int narrow = a_kind == RS_DY ? qm : a_kind == RS_U ? pm : b_kind == RS_U ? pm : b_kind == RS_DY ? qm : 1 << 30;
      const bool thin = !(a_kind == RS_STATE && b_kind == RS_STATE) && narrow <= 16;
      hipError_t er = sb     ? launch_outer_bf16(mp, rp, stream)
                      : ss   ? launch_outer_ss(mp, rp, stream)
                      : thin ? launch_outer_thin(mp, P.state_f64, rp, stream)
                             : launch_outer(mp, P.state_f64, rp, ty, stream);
      tl.done();
      return er;
    };
    if (grad_params) {
      // dC = sum dy x^T, dD = sum dy u^T per parameter set
      e = reduce(RS_DY, nullptr, nullptr, RS_STATE, xfinal, -1, tiles(qm, mp));
      if (e != hipSuccess) return hip_fail(e, "dC reduction launch");
      e = launch_sum(sj_dc + P.class_set_start[cl], ncs, qm * mp, 0, rp.partial, P.state_f64, G,
                     stream);
      if (e != hipSuccess) return hip_fail(e, "dC sum launch");
      e = reduce(RS_DY, nullptr, nullptr, RS_U, nullptr, -1, tiles(qm, pm));
      if (e != hipSuccess) return hip_fail(e, "dD reduction launch");
      e = launch_sum(sj_dd + P.class_set_start[cl], ncs, qm * pm, 0, rp.partial, P.state_f64, G,
                     stream);
      if (e != hipSuccess) return hip_fail(e, "dD sum launch");
    }
    // ---- reverse sweep, segment by segment ----
    for (int j = ml / c; j >= 0; --j) {
      const int kb = j * c;
      const int ke = std::min(kb + c - 1, ml);
      // recompute the stage inputs kb+1..ke from the checkpoint at kb
      prm.adjoint = 0;
      prm.flags = 0;
      prm.xin_first = nullptr;
      for (int k = kb; k < ke; ++k) {
        TimedLaunch tl(P, stream, 0);
        if (k + 1 <= J) {  // as in the forward: x^(k+1) by the input pass (the same bits)
          StageParams kp = prm;  // (prm.src may hold dy from an adjoint segment above)
          kp.src = u;
          kp.src_dtype = (int)u_dtype;
          kp.kry_override = k + 1;
          kp.xout = loc(k + 1);
          e = launch_krylov_res(mp, P.compute, kp,
                                reinterpret_cast<const ResRange*>(meta + P.m_ranges) + P.class_range_start[cl],
                                P.class_range_count[cl], stream);
        } else {
          prm.k = k;
          prm.xin = loc(k);
          prm.xout = loc(k + 1);
          prm.n_tiles = P.class_active[cl][k];
          e = launch_stage_any(P, cl, prm, stream);
        }
        if (e != hipSuccess) return hip_fail(e, "recompute stage launch");
        tl.done();
      }
      for (int k = ke; k >= kb; --k) {
        void* win = W[(k + 1) & 1];
        void* wout = W[k & 1];
        if (grad_params) {
          // dL/dP_k = sum_l g_l^(k+1) x_{l-2^k}^(k)^T
          e = reduce(RS_STATE, win, gfirst, RS_STATE, loc(k), k, tiles(mp, mp));
          if (e != hipSuccess) return hip_fail(e, "dP reduction launch");
          e = launch_sum(sj_dp + P.class_op_start[cl], nco, mp * mp, k, rp.partial, P.state_f64, G,
                         stream);
          if (e != hipSuccess) return hip_fail(e, "dP sum launch");
        }
        // g^(k) = g^(k+1) + shift_left(P_k^T g^(k+1)); at k = 0 also du
        prm.adjoint = 1;
        prm.k = k;
        prm.src = dy;
        prm.src_dtype = sdt;
        prm.dst = du;
        prm.flags = (du ? SF_EPILOGUE : 0) | SF_STORE_AT_EPI;
        prm.xin = win;
        prm.xin_first = gfirst;
        prm.xout = wout;
        prm.n_tiles = P.class_active[cl][k];
        TimedLaunch tl(P, stream, 1);
        e = launch_stage_any(P, cl, prm, stream);
        if (e != hipSuccess) return hip_fail(e, "adjoint stage launch");
        tl.done();
      }
    }
    prm.xin_first = nullptr;
    prm.src = u;
    prm.src_dtype = (int)u_dtype;
    if (grad_params) {
      // dBbar = sum g^(0) u^T per operator
      e = reduce(RS_STATE, W[0], nullptr, RS_U, nullptr, -1, tiles(mp, pm));
      if (e != hipSuccess) return hip_fail(e, "dBbar reduction launch");
      e = launch_sum(sj_dbb + P.class_op_start[cl], nco, mp * pm, 0, rp.partial, P.state_f64, G,
                     stream);
      if (e != hipSuccess) return hip_fail(e, "dBbar sum launch");
    }
  }
  if (dx0 || (x0 && grad_params)) {  // dL/dx_{-1} and the x_{-1} part of dL/dP_0, from g^(0) in W[0]
    unsigned char* meta = P.ws + P.r_meta.off;
    e = launch_x0_grads(P.state_f64 != 0, reinterpret_cast<const SeqDev*>(meta + P.m_seqs), P.n_seq,
                        reinterpret_cast<const OpDev*>(meta + P.m_ops), P.n_ops, P.at<double>(P.r_pw), x0, W[0], dx0,
                        x0 && grad_params ? G : nullptr, stream);
    if (e != hipSuccess) return hip_fail(e, "initial state gradient launch");
  }
  if (!grad_params) return SSM_OK;
  // ---- FP64: squaring adjoint, discretization adjoint, per-set sums ----
  for (size_t gi = 0; gi < P.bgroups.size(); ++gi) {
    const auto& gr = P.bgroups[gi];
    if (P.bkind[gi] == 0)
      e = launch_gemm_f64(bj_d + gr.first, gr.second, P.bdims[gi].first, P.bdims[gi].second,
                          stream);
    else
      e = launch_axpy(bj_d + gr.first, gr.second, P.bdims[gi].first, P.bdims[gi].second, stream);
    if (e != hipSuccess) return hip_fail(e, "FP64 adjoint launch");
  }
  if (P.disc == SSM_DISC_ZOH) {
    const GemmJob* zj = reinterpret_cast<const GemmJob*>(meta + P.m_zbjobs);
    for (size_t gi = 0; gi < P.zbgroups.size(); ++gi) {
      const auto& gr = P.zbgroups[gi];
      e = P.zbkind[gi] == 0 ? launch_gemm_f64(zj + gr.first, gr.second, P.zbdims[gi].first, P.zbdims[gi].second, stream)
                            : launch_axpy(zj + gr.first, gr.second, P.zbdims[gi].first, P.zbdims[gi].second, stream);
      if (e != hipSuccess) return hip_fail(e, "exponential adjoint launch");
    }
  }
  e = launch_scatter(reinterpret_cast<const ScatterJob*>(meta + P.m_scat), (int)P.scat.size(),
                     reinterpret_cast<const int32_t*>(meta + P.m_set_ops),
                     reinterpret_cast<const OpDev*>(meta + P.m_ops), G, grad_params, P.max_mp,
                     stream);
  if (e != hipSuccess) return hip_fail(e, "gradient scatter launch");
  return SSM_OK;
}

ssm_status ssm_cascade_backward(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                const void* dy, size_t dy_numel, void* du, double* grad_params,
                                size_t grad_numel, hipStream_t stream) {
  return backward_impl(plan, u, u_dtype, u_numel, nullptr, 0, dy, dy_numel, du, nullptr, 0, grad_params,
                       grad_numel, stream);
}

ssm_status ssm_cascade_backward_x0(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                   const void* x0, size_t x0_numel, const void* dy, size_t dy_numel, void* du,
                                   void* dx0, size_t dx0_numel, double* grad_params, size_t grad_numel,
                                   hipStream_t stream) {
  return backward_impl(plan, u, u_dtype, u_numel, x0, x0_numel, dy, dy_numel, du, dx0, dx0_numel, grad_params,
                       grad_numel, stream);
}

size_t ssm_cascade_param_grad_numel(ssm_plan plan) {
  if (!plan) return 0;
  return plan->grad_numel;
}

ssm_status ssm_cascade_get_power(ssm_plan plan, int32_t op, int32_t k, double* dst,
                                 hipStream_t stream) {
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (op < 0 || op >= plan->n_ops) return fail(SSM_E_INVALID, "operator %d out of range", op);
  const OpDev& o = plan->ops[op];
  if (k < 0 || k > o.N) return fail(SSM_E_INVALID, "power index %d outside 0..%d", k, o.N);
  if (!dst) return fail(SSM_E_INVALID, "dst is NULL");
  const double* srcp = plan->at<double>(plan->r_pw) + o.pw + (int64_t)k * o.mp * o.mp;
  HIP_TRY(hipMemcpy2DAsync(dst, (size_t)o.m * 8, srcp, (size_t)o.mp * 8, (size_t)o.m * 8, o.m,
                           hipMemcpyDeviceToDevice, stream),
          "power copy");
  return SSM_OK;
}

ssm_status ssm_cascade_get_bbar(ssm_plan plan, int32_t op, double* dst, hipStream_t stream) {
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (op < 0 || op >= plan->n_ops) return fail(SSM_E_INVALID, "operator %d out of range", op);
  if (!dst) return fail(SSM_E_INVALID, "dst is NULL");
  const OpDev& o = plan->ops[op];
  const double* srcp = plan->at<double>(plan->r_bbar) + o.bbar;
  HIP_TRY(hipMemcpyAsync(dst, srcp, (size_t)o.m * o.p * 8, hipMemcpyDeviceToDevice, stream),
          "Bbar copy");
  return SSM_OK;
}

ssm_status ssm_cascade_device_status(ssm_plan plan, hipStream_t stream) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  ssm_plan_s& P = *plan;
  HIP_TRY(hipStreamSynchronize(stream), "synchronization");
  if (P.launch != SSM_LAUNCH_PERSISTENT) return SSM_OK;
  int32_t* flag = reinterpret_cast<int32_t*>(P.ws + P.r_meta.off + P.m_counters) + P.n_counters;
  int32_t h = 0;
  HIP_TRY(hipMemcpy(&h, flag, sizeof h, hipMemcpyDeviceToHost), "give-up flag read");
  if (h != 0)
    return fail(SSM_E_HIP, "a persistent launch gave up waiting for the items it depends on "
                           "(spin limit %d); its output is not valid",
                P.spin_limit > 0 ? P.spin_limit : (int)kPersistSpinLimit);
  return SSM_OK;
}

ssm_status ssm_cascade_plan_stages(ssm_plan plan, int32_t* N, int32_t n) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (!N || n != plan->n_seq) return fail(SSM_E_INVALID, "N must hold the plan's %d sequences", plan->n_seq);
  for (int i = 0; i < n; ++i) N[i] = plan->desc[i].N;
  return SSM_OK;
}

ssm_status ssm_cascade_plan_info(ssm_plan plan, ssm_plan_info* info) {
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (!info) return fail(SSM_E_INVALID, "info is NULL");
  info->n_seq = plan->n_seq;
  info->n_ops = plan->n_ops;
  info->compute = plan->compute;
  info->max_stage = plan->max_last;
  info->total_steps = plan->total_steps;
  info->stage_flops = plan->stage_flops;
  info->io_flops = plan->io_flops;
  info->stage_bytes = plan->stage_bytes;
  info->stage_launches = plan->stage_launches;
  info->launch = plan->launch;
  // the tiled kernel runs the items of a persistent launch unless the resident items do
  info->stage_kernel = plan->launch == SSM_LAUNCH_PERSISTENT && !plan->persist_res
                           ? (int32_t)SSM_STAGE_TILED
                           : plan->stage_kernel;
  info->input_stages = plan->max_kry;
  for (int c = 0; c < 4; ++c) info->tile_rows[c] = plan->class_bm[c];
  info->persistent_grid = plan->persistent_grid;
  info->persistent_items = (int64_t)(plan->persist_res ? plan->ritems.size() : plan->items.size());
  info->pair_launches = plan->pair_launches;
  info->pair_bytes = plan->pair_bytes;
  info->pair_flops = plan->pair_flops;
  info->state_dtype = plan->state_bf16 ? SSM_BF16 : plan->state_f64 ? SSM_F64 : SSM_F32;
  info->fold_launches = plan->fold_launches;
  info->fold_bytes = plan->fold_bytes;
  info->fold_flops = plan->fold_flops;
  info->fold_stages = 0;
  for (int c = 0; c < 4; ++c) info->fold_stages = std::max(info->fold_stages, plan->fold_s[c]);
  for (int f : plan->seq_fold_s) info->fold_stages = std::max(info->fold_stages, f);
  info->lower_ops = 0;
  for (const OpDev& o : plan->ops) info->lower_ops += o.lower != 0;
  info->plr_stages = plan->plr_stages;
  info->plr_reserved = 0;
  info->lower_reserved = 0;
  info->plr_flops = plan->plr_flops;
  info->plr_dense_flops = plan->plr_dense_flops;
  return SSM_OK;
}

ssm_status ssm_cascade_plr_ranks(ssm_plan plan, int32_t op, int32_t k, int32_t* ranks, int32_t n,
                                 int32_t* used) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (!ranks || !used || n < kPlrRankSlots) return fail(SSM_E_INVALID, "ranks must hold %d entries", kPlrRankSlots);
  if (op < 0 || op >= plan->n_ops) return fail(SSM_E_INVALID, "op %d outside 0..%d", op, plan->n_ops - 1);
  const OpDev& o = plan->ops[op];
  if (k < 0 || k > o.N) return fail(SSM_E_INVALID, "k %d outside 0..%d", k, o.N);
  if (plan->plr_digits <= 0 || plan->plr_rank_off.empty() || plan->plr_rank_off[op] < 0)
    return fail(SSM_E_UNSUPPORTED, "operator %d has no PLR powers (plr_digits 0, padded m 32 or no eligible stage)",
                op);
  const int c = class_of(o.mp);
  for (int i = 0; i < kPlrRankSlots; ++i)
    ranks[i] = plan->plr_ranks_host[(size_t)plan->plr_rank_off[op] + (size_t)k * kPlrRankSlots + i];
  *used = k < (int)plan->plr_use[c].size() ? plan->plr_use[c][k] : 0;
  return SSM_OK;
}

ssm_status ssm_cascade_timing_enable(ssm_plan plan, int32_t enable) {
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  plan->timing = enable != 0;
  return SSM_OK;
}

ssm_status ssm_cascade_timing_read(ssm_plan plan, int32_t kind, int64_t* launches,
                                   double* total_ms) {
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (!launches || !total_ms) return fail(SSM_E_INVALID, "NULL output");
  int64_t n = 0;
  double ms = 0.0;
  std::vector<TimingRec> keep;
  for (TimingRec& r : plan->trec) {
    if (r.kind != kind) {
      keep.push_back(r);
      continue;
    }
    HIP_TRY(hipEventSynchronize(r.b), "event synchronize");
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b), "event elapsed");
    ms += t;
    ++n;
    plan->event_pool.push_back(r.a);
    plan->event_pool.push_back(r.b);
  }
  plan->trec.swap(keep);
  *launches = n;
  *total_ms = ms;
  return SSM_OK;
}

}  // extern "C"

struct ssm_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

template <typename F>
ssm_status capture(ssm_plan plan, hipStream_t stream, ssm_graph* out, F&& call) {
  if (!out) return fail(SSM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  if (!stream) return fail(SSM_E_INVALID, "graph capture needs a stream other than 0");
  const bool timing = plan->timing;
  plan->timing = false;
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    plan->timing = timing;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  ssm_status st = call();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(stream, &g);
  plan->timing = timing;
  if (st != SSM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  ssm_graph_s* G = new (std::nothrow) ssm_graph_s();
  if (!G) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return fail(SSM_E_INVALID, "out of host memory");
  }
  G->graph = g;
  G->exec = x;
  *out = G;
  return SSM_OK;
}

}  // namespace

extern "C" {

ssm_status ssm_cascade_graph_apply(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                   size_t u_numel, void* y, size_t y_numel, hipStream_t stream,
                                   ssm_graph* out) {
  return capture(plan, stream, out, [&]() {
    return ssm_cascade_apply(plan, u, u_dtype, u_numel, y, y_numel, stream);
  });
}

ssm_status ssm_cascade_graph_backward(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                      size_t u_numel, const void* dy, size_t dy_numel, void* du,
                                      double* grad_params, size_t grad_numel, hipStream_t stream,
                                      ssm_graph* out) {
  return capture(plan, stream, out, [&]() {
    return ssm_cascade_backward(plan, u, u_dtype, u_numel, dy, dy_numel, du, grad_params,
                                grad_numel, stream);
  });
}

ssm_status ssm_cascade_graph_launch(ssm_graph graph, hipStream_t stream) {
  if (!graph) return fail(SSM_E_INVALID, "graph is NULL");
  HIP_TRY(hipGraphLaunch(graph->exec, stream), "hipGraphLaunch");
  return SSM_OK;
}

ssm_status ssm_cascade_graph_destroy(ssm_graph graph) {
  if (!graph) return SSM_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return SSM_OK;
}

ssm_status ssm_cascade_destroy(ssm_plan plan) {
  if (!plan) return SSM_OK;
  for (TimingRec& r : plan->trec) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : plan->event_pool) (void)hipEventDestroy(e);
  delete plan;
  return SSM_OK;
}

}  // extern "C"
