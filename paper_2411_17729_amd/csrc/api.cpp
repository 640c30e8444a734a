// Host side of the C ABI declared in include/ssm_cascade.h: argument
// validation, operator de-duplication, workspace carving, device tables and
// the launch sequences of prepare / apply / recursion / backward.
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
#include "ssm_internal.h"

using namespace ssmc;

namespace {

thread_local std::string g_last_error;

ssm_status fail(ssm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

ssm_status hip_fail(hipError_t e, const char* what) {
  return fail(SSM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                    \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

inline int pad_m(int m) { return m <= 32 ? 32 : m <= 64 ? 64 : m <= 128 ? 128 : 256; }
inline int class_of(int mp) { return mp == 32 ? 0 : mp == 64 ? 1 : mp == 128 ? 2 : 3; }
constexpr int kClassMp[4] = {32, 64, 128, 256};

inline size_t dt_size(int dt) { return dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : 2; }

// Last stage index that changes anything: stage k updates rows 2^k..L-1.
inline int last_stage(int N, int64_t L) {
  if (L <= 1) return 0;
  int k = 0;
  while (k < N && ((int64_t)1 << (k + 1)) <= L - 1) ++k;
  return k;
}

struct Region {
  size_t off = 0, bytes = 0;
};

struct TimingRec {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct ssm_plan_s {
  // configuration
  int n_seq = 0, n_ops = 0, n_sets = 0;
  int compute = DT_F32;  // DT_* of the stage operands
  int state_f64 = 0;     // state / io element is double
  int disc = 0;
  int with_backward = 0, ckpt_every = 1;
  int max_last = 0, max_mp = 32, max_N = 0;
  // host copies
  std::vector<ssm_seq_desc> desc;
  std::vector<SeqDev> seqs;
  std::vector<OpDev> ops;
  std::vector<OpSrc> src;
  std::vector<Tile> tiles;
  int class_tile_start[4] = {0, 0, 0, 0};
  int class_tile_count[4] = {0, 0, 0, 0};
  int class_max_last[4] = {-1, -1, -1, -1};
  std::vector<int> class_active[4];  // tiles active at stage k (prefix length)
  std::vector<int> set_m, set_p, set_q;
  int64_t sum_rows[4] = {0, 0, 0, 0};
  // workspace
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  Region r_meta, r_pw, r_pc, r_bbar, r_minv, r_small, r_aug, r_nmat, r_bsc, r_x0, r_x1;
  size_t m_seqs = 0, m_ops = 0, m_src = 0, m_tiles = 0, m_status = 0, m_jobs = 0;
  std::vector<GemmJob> jobs;            // prepare jobs, in launch order
  std::vector<std::pair<int, int>> job_groups;  // (start, count) per launch
  std::vector<std::pair<int, int>> job_dims;    // (max M, max N) per launch
  size_t meta_bytes = 0;
  std::vector<unsigned char> meta_host;
  // info
  double stage_flops = 0, io_flops = 0, stage_bytes = 0;
  int64_t total_steps = 0, stage_launches = 0;
  // timing
  bool timing = false;
  std::vector<TimingRec> trec;
  std::vector<hipEvent_t> event_pool;  // events reused across timing reads

  template <typename T>
  T* at(const Region& r) const {
    return reinterpret_cast<T*>(ws + r.off);
  }
  size_t x_elem() const { return state_f64 ? 8 : 4; }
};

namespace {

// ---------------------------------------------------------------------------
// validation and planning (host only; shared by workspace_bytes and prepare)
// ---------------------------------------------------------------------------
ssm_status validate_seqs(const ssm_seq_desc* seqs, int32_t n_seq) {
  if (!seqs) return fail(SSM_E_INVALID, "seqs is NULL");
  if (n_seq <= 0) return fail(SSM_E_INVALID, "n_seq must be positive (got %d)", n_seq);
  for (int i = 0; i < n_seq; ++i) {
    const ssm_seq_desc& d = seqs[i];
    if (d.m < 1 || d.m > 256)
      return fail(SSM_E_UNSUPPORTED, "seq %d: m=%d outside 1..256", i, d.m);
    if (d.p < 1 || d.p > d.m) return fail(SSM_E_INVALID, "seq %d: p=%d outside 1..m", i, d.p);
    if (d.q < 1 || d.q > d.m) return fail(SSM_E_INVALID, "seq %d: q=%d outside 1..m", i, d.q);
    if (d.N < 0 || d.N > 62) return fail(SSM_E_INVALID, "seq %d: N=%d outside 0..62", i, d.N);
    if (d.L < 1 || d.L > ((int64_t)1 << 31) - 1)
      return fail(SSM_E_INVALID, "seq %d: L=%lld outside 1..2^31-1", i, (long long)d.L);
    if (d.param_set < 0) return fail(SSM_E_INVALID, "seq %d: negative param_set", i);
    if (d.reserved != 0) return fail(SSM_E_INVALID, "seq %d: reserved must be 0", i);
    if (d.u_offset < 0 || d.y_offset < 0)
      return fail(SSM_E_INVALID, "seq %d: negative offset", i);
  }
  return SSM_OK;
}

// Builds sequences, operators, tiles, info and the workspace layout.
ssm_status build_plan(ssm_plan_s& P, const ssm_seq_desc* seqs, int32_t n_seq, ssm_disc disc,
                      ssm_dtype compute, int32_t with_backward, int32_t ckpt_every) {
  ssm_status st = validate_seqs(seqs, n_seq);
  if (st != SSM_OK) return st;
  if (disc != SSM_DISC_TRAPEZOID && disc != SSM_DISC_GIVEN)
    return fail(SSM_E_INVALID, "unknown discretization %d", (int)disc);
  if (compute != SSM_F64 && compute != SSM_F32 && compute != SSM_BF16)
    return fail(SSM_E_INVALID, "unknown compute dtype %d", (int)compute);
  if (ckpt_every < 0) return fail(SSM_E_INVALID, "ckpt_every must be >= 0");
  P.n_seq = n_seq;
  P.compute = (int)compute;
  P.state_f64 = compute == SSM_F64;
  P.disc = (int)disc;
  P.with_backward = with_backward != 0;
  P.desc.assign(seqs, seqs + n_seq);

  // operators: distinct (param_set, delta) in order of first appearance
  std::map<std::pair<int, uint64_t>, int> key2op;
  P.seqs.resize(n_seq);
  std::vector<int> op_last;
  int n_sets = 0;
  for (int i = 0; i < n_seq; ++i) {
    const ssm_seq_desc& d = seqs[i];
    if (disc == SSM_DISC_TRAPEZOID && !(d.delta > 0.0 && std::isfinite(d.delta)))
      return fail(SSM_E_INVALID, "seq %d: delta must be positive and finite", i);
    uint64_t dbits = 0;
    if (disc == SSM_DISC_TRAPEZOID) std::memcpy(&dbits, &d.delta, 8);
    auto key = std::make_pair(d.param_set, dbits);
    int op;
    auto it = key2op.find(key);
    const int lst = last_stage(d.N, d.L);
    if (it == key2op.end()) {
      op = (int)P.ops.size();
      key2op[key] = op;
      OpDev o{};
      o.m = d.m;
      o.mp = pad_m(d.m);
      o.p = d.p;
      o.q = d.q;
      o.set = d.param_set;
      o.delta = disc == SSM_DISC_TRAPEZOID ? d.delta : 0.0;
      o.N = lst;
      P.ops.push_back(o);
    } else {
      op = it->second;
      OpDev& o = P.ops[op];
      if (o.m != d.m || o.p != d.p || o.q != d.q)
        return fail(SSM_E_INVALID, "seq %d: sizes differ from another sequence of set %d", i,
                    d.param_set);
      o.N = std::max(o.N, lst);
    }
    n_sets = std::max(n_sets, d.param_set + 1);
    SeqDev& s = P.seqs[i];
    s.L = d.L;
    s.u_off = d.u_offset;
    s.y_off = d.y_offset;
    s.op = op;
    s.last = lst;
    s.p = d.p;
    s.q = d.q;
  }
  // sets shared by several operators must agree on sizes
  P.set_m.assign(n_sets, -1);
  P.set_p.assign(n_sets, -1);
  P.set_q.assign(n_sets, -1);
  for (const OpDev& o : P.ops) {
    if (P.set_m[o.set] >= 0 &&
        (P.set_m[o.set] != o.m || P.set_p[o.set] != o.p || P.set_q[o.set] != o.q))
      return fail(SSM_E_INVALID, "parameter set %d used with different sizes", o.set);
    P.set_m[o.set] = o.m;
    P.set_p[o.set] = o.p;
    P.set_q[o.set] = o.q;
  }
  P.n_sets = n_sets;
  P.n_ops = (int)P.ops.size();

  // tiles per size class, sequences ordered by last stage (descending) so the
  // tiles active at stage k form a prefix
  for (int c = 0; c < 4; ++c) {
    std::vector<int> ids;
    for (int i = 0; i < n_seq; ++i)
      if (P.ops[P.seqs[i].op].mp == kClassMp[c]) ids.push_back(i);
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int a, int b) { return P.seqs[a].last > P.seqs[b].last; });
    const int bm = stage_bm(kClassMp[c], P.compute);
    P.class_tile_start[c] = (int)P.tiles.size();
    int ml = -1;
    for (int i : ids) {
      for (int64_t r0 = 0; r0 < P.seqs[i].L; r0 += bm) P.tiles.push_back(Tile{i, (int32_t)r0});
      ml = std::max(ml, P.seqs[i].last);
    }
    P.class_tile_count[c] = (int)P.tiles.size() - P.class_tile_start[c];
    P.class_max_last[c] = ml;
    P.class_active[c].assign(ml + 1, 0);
    for (int kk = 0; kk <= ml; ++kk) {
      int cnt = 0;
      for (int ti = P.class_tile_start[c]; ti < (int)P.tiles.size(); ++ti)
        if (P.seqs[P.tiles[ti].seq].last >= kk) ++cnt;
      P.class_active[c][kk] = cnt;
    }
  }

  // state offsets, sizes, info
  int64_t xrows = 0;
  P.max_last = 0;
  P.max_mp = 32;
  P.stage_flops = P.io_flops = P.stage_bytes = 0;
  P.total_steps = 0;
  for (int i = 0; i < n_seq; ++i) {
    SeqDev& s = P.seqs[i];
    const OpDev& o = P.ops[s.op];
    s.x_off = xrows * o.mp;  // filled per class below; temporary
    P.max_last = std::max(P.max_last, s.last);
    P.max_mp = std::max(P.max_mp, o.mp);
    P.total_steps += s.L;
    P.io_flops += 2.0 * o.m * s.p * s.L + 2.0 * s.q * (o.m + s.p) * s.L;
    for (int kk = 0; kk <= s.last; ++kk) {
      const int64_t sh = (int64_t)1 << kk;
      if (sh < s.L) {
        P.stage_flops += 2.0 * o.m * o.m * (double)(s.L - sh);
      }
    }
    xrows += s.L;
  }
  // x offsets in elements: sequences back to back, each L x mp
  int64_t xoff = 0;
  for (int i = 0; i < n_seq; ++i) {
    SeqDev& s = P.seqs[i];
    s.x_off = xoff;
    xoff += s.L * (int64_t)P.ops[s.op].mp;
  }
  // algorithmic HBM bytes of the stage launches: per stage and row, read the
  // row and (for rows with a partner) the shifted partner, and write the row
  // (state element size); the last stage writes y instead of the state.
  const double xe = (double)P.x_elem();
  P.stage_launches = 0;
  for (int c = 0; c < 4; ++c) P.stage_launches += P.class_max_last[c] + 1;
  for (int i = 0; i < n_seq; ++i) {
    const SeqDev& s = P.seqs[i];
    const int m = P.ops[s.op].m;
    for (int kk = 0; kk <= s.last; ++kk) {
      const double in_row = (double)m * xe;
      const double out_row = kk == s.last ? (double)s.q * xe : (double)m * xe;
      const int64_t sh = (int64_t)1 << kk;
      const double upd_rows = sh < s.L ? (double)(s.L - sh) : 0.0;
      P.stage_bytes += s.L * (in_row + out_row) + upd_rows * in_row;
    }
  }

  P.max_N = 0;
  for (const OpDev& o : P.ops) P.max_N = std::max(P.max_N, o.N);
  int nst = P.max_last + 1;
  P.ckpt_every = ckpt_every == 0 ? (int)std::ceil(std::sqrt((double)nst)) : ckpt_every;
  if (P.ckpt_every < 1) P.ckpt_every = 1;

  // ---- workspace layout ----
  const size_t ce = dt_size(P.compute);
  size_t n_pw = 0, n_pc = 0, n_bbar = 0, n_minv = 0, n_small = 0, n_aug = 0, n_nmat = 0,
         n_bsc = 0;
  for (OpDev& o : P.ops) {
    const size_t mm = (size_t)o.mp * o.mp;
    o.pw = (int64_t)n_pw;
    n_pw += (size_t)(o.N + 1) * mm;
    o.pc = (int64_t)n_pc;
    n_pc += (size_t)(o.N + 1) * mm;
    if (P.with_backward) {
      o.pct = (int64_t)n_pc;
      n_pc += (size_t)(o.N + 1) * mm;
    } else {
      o.pct = -1;
    }
    o.bbar = (int64_t)n_bbar;
    n_bbar += (size_t)o.mp * o.p;
    o.minv = (int64_t)n_minv;
    n_minv += mm;
    o.bin = (int64_t)n_small;
    n_small += (size_t)o.mp * o.p;
    o.bt = (int64_t)n_small;
    n_small += (size_t)o.mp * o.p;
    o.cout = (int64_t)n_small;
    n_small += (size_t)o.q * o.mp;
    o.ct = (int64_t)n_small;
    n_small += (size_t)o.q * o.mp;
    o.dmat = (int64_t)n_small;
    n_small += (size_t)o.q * o.p;
    o.dt = (int64_t)n_small;
    n_small += (size_t)o.q * o.p;
    if (disc == SSM_DISC_TRAPEZOID) {
      o.sc_aug = (int64_t)n_aug;
      n_aug += 2 * mm;
      o.sc_n = (int64_t)n_nmat;
      n_nmat += mm;
      o.sc_b = (int64_t)n_bsc;
      n_bsc += (size_t)o.mp * o.p;
    } else {
      o.sc_aug = o.sc_n = o.sc_b = -1;
    }
  }
  // prepare GEMM jobs (pointers are patched once the workspace is known)
  P.jobs.clear();
  P.job_groups.clear();
  P.job_dims.clear();

  // meta region: tables
  size_t off = 0;
  P.m_seqs = off;
  off = align_up(off + sizeof(SeqDev) * P.seqs.size());
  P.m_ops = off;
  off = align_up(off + sizeof(OpDev) * P.ops.size());
  P.m_src = off;
  off = align_up(off + sizeof(OpSrc) * P.ops.size());
  P.m_tiles = off;
  off = align_up(off + sizeof(Tile) * std::max<size_t>(1, P.tiles.size()));
  P.m_status = off;
  off = align_up(off + 16);
  // jobs: 2 per operator (discretization) + one per operator and squaring
  size_t n_jobs = 2 * P.ops.size();
  for (const OpDev& o : P.ops) n_jobs += (size_t)o.N;
  P.m_jobs = off;
  off = align_up(off + sizeof(GemmJob) * std::max<size_t>(1, n_jobs));
  P.meta_bytes = off;

  size_t cur = 0;
  auto take = [&](Region& r, size_t bytes) {
    r.off = cur;
    r.bytes = bytes;
    cur = align_up(cur + bytes);
  };
  take(P.r_meta, P.meta_bytes);
  take(P.r_pw, n_pw * 8);
  take(P.r_pc, n_pc * ce);
  take(P.r_bbar, n_bbar * 8);
  take(P.r_minv, n_minv * 8);
  take(P.r_small, n_small * P.x_elem());
  take(P.r_aug, n_aug * 8);
  take(P.r_nmat, n_nmat * 8);
  take(P.r_bsc, n_bsc * 8);
  take(P.r_x0, (size_t)xoff * P.x_elem());
  take(P.r_x1, (size_t)xoff * P.x_elem());
  P.ws_bytes = cur;
  return SSM_OK;
}

// Records an event pair around a launch when timing is on.
struct TimedLaunch {
  ssm_plan_s& P;
  hipStream_t s;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(ssm_plan_s& P_, hipStream_t s_, int kind_) : P(P_), s(s_), kind(kind_) {
    if (P.timing) {
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
    if (P.timing) {
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
                                   int32_t ckpt_every) {
  ssm_plan_s P;
  if (build_plan(P, seqs, n_seq, disc, compute, with_backward, ckpt_every) != SSM_OK) return 0;
  return P.ws_bytes;
}

ssm_status ssm_cascade_prepare(const ssm_seq_desc* seqs, int32_t n_seq, const ssm_params* sets,
                               int32_t n_sets, ssm_disc disc, ssm_dtype compute,
                               int32_t with_backward, int32_t ckpt_every, void* ws,
                               size_t ws_bytes, hipStream_t stream, ssm_plan* out) {
  g_last_error.clear();
  if (!out) return fail(SSM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!sets) return fail(SSM_E_INVALID, "sets is NULL");
  if (!ws) return fail(SSM_E_INVALID, "workspace is NULL");
  ssm_plan_s* P = new (std::nothrow) ssm_plan_s();
  if (!P) return fail(SSM_E_INVALID, "out of host memory");
  ssm_status st = build_plan(*P, seqs, n_seq, disc, compute, with_backward, ckpt_every);
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
  if (disc == SSM_DISC_TRAPEZOID) {
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
  }
  for (int kk = 0; kk < P->max_N; ++kk) {  // P_{k+1} = P_k P_k
    int start = (int)J.size(), mx = 0;
    for (const OpDev& o : P->ops) {
      if (o.N <= kk) continue;
      const int64_t mm = (int64_t)o.mp * o.mp;
      double* Pk = pw + o.pw + kk * mm;
      J.push_back(GemmJob{Pk, Pk, Pk + mm, o.mp, o.mp, o.mp, o.mp, o.mp, o.mp, 0, 0, 1.0, 0.0});
      mx = std::max(mx, o.mp);
    }
    P->job_groups.push_back({start, (int)J.size() - start});
    P->job_dims.push_back({mx, mx});
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
  e = launch_disc_setup(ops_d, P->n_ops, src_d, given, P->at<double>(P->r_aug), nmat, bsc, pw,
                        bbar, P->max_mp, stream);
  if (e != hipSuccess) return bail(hip_fail(e, "discretization setup launch"));
  size_t g = 0;
  if (!given) {
    e = launch_gauss_jordan(ops_d, P->n_ops, P->at<double>(P->r_aug), minv, status_d, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "Gauss-Jordan launch"));
    const auto& grp = P->job_groups[g];
    e = launch_gemm_f64(jobs_d + grp.first, grp.second, P->job_dims[g].first,
                        P->job_dims[g].second, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "discretization GEMM launch"));
    ++g;
  }
  for (; g < P->job_groups.size(); ++g) {
    const auto& grp = P->job_groups[g];
    e = launch_gemm_f64(jobs_d + grp.first, grp.second, P->job_dims[g].first,
                        P->job_dims[g].second, stream);
    if (e != hipSuccess) return bail(hip_fail(e, "squaring GEMM launch"));
  }
  e = launch_pack(ops_d, P->n_ops, src_d, pw, bbar, P->ws + P->r_pc.off, P->compute,
                  P->with_backward, P->ws + P->r_small.off, P->state_f64, P->max_mp, P->max_N,
                  stream);
  if (e != hipSuccess) return bail(hip_fail(e, "pack launch"));
  int status_h[4] = {0, 0, 0, 0};
  e = hipMemcpyAsync(status_h, status_d, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return bail(hip_fail(e, "status read"));
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bail(hip_fail(e, "prepare synchronization"));
  if (status_h[0] != 0)
    return bail(fail(SSM_E_NUMERIC, "I - delta/2 A is singular to working precision"));
  *out = P;
  return SSM_OK;
}

ssm_status ssm_cascade_apply(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                             void* y, size_t y_numel, hipStream_t stream) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  ssm_plan_s& P = *plan;
  ssm_status st = check_io(P, u, u_dtype, u_numel, y, y_numel, "y");
  if (st != SSM_OK) return st;
  for (int c = 0; c < 4; ++c) {
    if (P.class_tile_count[c] == 0) continue;
    StageParams prm = base_params(P, c);
    prm.src = u;
    prm.src_dtype = (int)u_dtype;
    prm.dst = y;
    prm.adjoint = 0;
    // V^(0) = Bbar U into the first state buffer
    prm.xout = P.ws + P.r_x0.off;
    prm.n_tiles = P.class_tile_count[c];
    hipError_t e = launch_project(kClassMp[c], P.state_f64, prm, stream);
    if (e != hipSuccess) return hip_fail(e, "projection launch");
    prm.flags = SF_EPILOGUE;
    for (int kk = 0; kk <= P.class_max_last[c]; ++kk) {
      prm.k = kk;
      prm.xin = P.ws + ((kk & 1) ? P.r_x1.off : P.r_x0.off);
      prm.xout = P.ws + ((kk & 1) ? P.r_x0.off : P.r_x1.off);
      prm.n_tiles = P.class_active[c][kk];
      TimedLaunch tl(P, stream, 0);
      e = launch_stage(kClassMp[c], P.compute, prm, stream);
      if (e != hipSuccess) return hip_fail(e, "stage launch");
      tl.done();
    }
  }
  return SSM_OK;
}

ssm_status ssm_cascade_recursion(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                 size_t u_numel, void* y, size_t y_numel, hipStream_t stream) {
  g_last_error.clear();
  if (!plan) return fail(SSM_E_NOT_PREPARED, "plan is NULL");
  ssm_plan_s& P = *plan;
  ssm_status st = check_io(P, u, u_dtype, u_numel, y, y_numel, "y");
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
    hipError_t e = launch_stage(kClassMp[c], P.compute, prm, stream);
    if (e != hipSuccess) return hip_fail(e, "projection launch");
  }
  return SSM_OK;
}

ssm_status ssm_cascade_backward(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                const void* dy, size_t dy_numel, void* du, double* grad_params,
                                size_t grad_numel, hipStream_t stream) {
  (void)plan; (void)u; (void)u_dtype; (void)u_numel; (void)dy; (void)dy_numel; (void)du;
  (void)grad_params; (void)grad_numel; (void)stream;
  return fail(SSM_E_UNSUPPORTED, "backward is not built yet");
}

size_t ssm_cascade_param_grad_numel(ssm_plan plan) {
  if (!plan) return 0;
  size_t n = 0;
  for (int s = 0; s < plan->n_sets; ++s) {
    const size_t m = plan->set_m[s] < 0 ? 0 : plan->set_m[s];
    const size_t p = plan->set_p[s] < 0 ? 0 : plan->set_p[s];
    const size_t q = plan->set_q[s] < 0 ? 0 : plan->set_q[s];
    n += m * m + m * p + q * m + q * p;
  }
  return n;
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
