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
#include "plr.h"

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
// exponential discretization: Taylor terms after scaling to 1-norm <= 1/2
// (remainder below 0.5^19 e^0.5 / 19! < 2e-23), and the most squarings
constexpr int kZohTaylor = 18;
constexpr int kZohMaxSq = 60;

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
  int state_bf16 = 0;    // the forward apply keeps the state between passes in BF16
  int static_state = 0;  // the workspace holds no state buffers (ssm_cascade_apply_noalloc only)
  int final_state = 0;   // the forward apply leaves each sequence's final state in the buffers
  size_t x_buf_bytes = 0;  // bytes of one state buffer
  int disc = 0;
  int with_backward = 0, ckpt_every = 1;
  int max_last = 0, max_mp = 32, max_N = 0;
  int min_mp = 32;  // smallest padded state size (ssm_tuning.min_padded_m)
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
  // automatic N: the Frobenius norms of every operator's powers, (N + 1) per
  // operator in operator order (only while choosing N)
  Region r_norms;
  int64_t n_norms = 0;
  // exponential discretization: per-operator scratch, the identity (z_nid x
  // z_nid) and the norms (element offsets in r_zoh); its jobs, made once the
  // norms are read back, in a meta area of z_cap jobs at m_zjobs
  Region r_zoh;
  int64_t z_id = 0, z_norm = 0;
  int z_nid = 0;
  size_t m_zjobs = 0, z_cap = 0;
  // its adjoint (backward plans): jobs at m_zbjobs (capacity zb_cap), groups
  std::vector<GemmJob> zbjobs;
  std::vector<std::pair<int, int>> zbgroups, zbdims;
  std::vector<int> zbkind;
  size_t m_zbjobs = 0, zb_cap = 0;
  size_t m_seqs = 0, m_ops = 0, m_src = 0, m_tiles = 0, m_status = 0, m_jobs = 0, m_tri = 0, m_tri_scale = 0;
  std::vector<GemmJob> jobs;            // prepare jobs, in launch order
  std::vector<std::pair<int, int>> job_groups;  // (start, count) per launch
  std::vector<std::pair<int, int>> job_dims;    // (max M, max N) per launch
  std::vector<int> job_kind;                    // 0: GEMM, 1: axpy
  size_t meta_bytes = 0;
  std::vector<unsigned char> meta_host;
  // info
  double stage_flops = 0, io_flops = 0, stage_bytes = 0;
  int64_t total_steps = 0, stage_launches = 0;
  // timing
  bool timing = false;
  std::vector<TimingRec> trec;
  std::vector<hipEvent_t> event_pool;  // events reused across timing reads
  // tuning
  int launch = SSM_LAUNCH_PER_STAGE;
  int stage_kernel = SSM_STAGE_TILED;
  int class_bm[4] = {0, 0, 0, 0};
  int max_kry = 0;                  // leading stages folded into the input pass
  // split input pass: row ranges per class (empty where the resident pass runs)
  std::vector<ResRange> input_units;
  int class_input_start[4] = {0, 0, 0, 0}, class_input_count[4] = {0, 0, 0, 0};
  size_t class_input_lds[4] = {0, 0, 0, 0};
  int class_input_p[4] = {0, 0, 0, 0}, class_input_kdim[4] = {0, 0, 0, 0};
  size_t m_input = 0;
  int class_min_kry[4] = {0, 0, 0, 0};
  int class_all_kry[4] = {0, 0, 0, 0};  // every sequence of the class is folded
  Region r_kw;
  // resident-power stage kernel: row ranges per class, longest-running first
  std::vector<ResRange> ranges;
  int class_range_start[4] = {0, 0, 0, 0}, class_range_count[4] = {0, 0, 0, 0};
  std::vector<int> class_range_active[4];
  std::vector<int> class_final[4];  // sequences whose last stage is k
  size_t m_ranges = 0;
  // chain stage kernel: work units per class and stage (empty where unused)
  std::vector<ChainUnit> chain_units;
  std::vector<int> chain_start[4], chain_count[4], chain_T[4];
  size_t m_chain = 0;
  // stage pairs of the forward apply: units per class at the pair's first stage
  std::vector<PairUnit> pair_units;
  std::vector<int> pair_start[4], pair_count[4], pair_tail[4];
  std::vector<size_t> pair_lds_bytes[4];
  size_t m_pair = 0;
  int64_t pair_launches = 0;
  double pair_bytes = 0, pair_flops = 0;
  // output pass with the last stages folded in: per class the first folded
  // stage and their number (0: none), workgroup units, LDS bytes
  int fold_k0[4] = {0, 0, 0, 0}, fold_s[4] = {0, 0, 0, 0};
  bool fold_wide[4] = {false, false, false, false};  // six stages, paired lags, lags split over waves
  // classes whose sequences end at different stages (ragged batches): each
  // sequence folds its own last seq_fold_s stages from seq_fold_k0 on, after
  // stage pairs from the input pass up to there; the folds run as launches
  // grouped by kernel, depth and the state buffer holding their input
  bool fold_mixed[4] = {false, false, false, false};
  std::vector<int> seq_fold_s, seq_fold_k0;
  struct FoldLaunch {
    int c, wide, s, buf, start, count, max_p;
    bool q4;
    size_t lds;
  };
  std::vector<FoldLaunch> mixed_folds;
  std::vector<FoldUnit> fold_units;
  int fold_start[4] = {0, 0, 0, 0}, fold_count[4] = {0, 0, 0, 0};
  size_t fold_lds_bytes[4] = {0, 0, 0, 0};
  int fold_max_p[4] = {0, 0, 0, 0};  // widest input of the class's folded sequences
  bool fold_q4[4] = {false, false, false, false};  // every q and y offset of the class a multiple of 4
  size_t m_fold = 0;
  int64_t fold_launches = 0;
  double fold_bytes = 0, fold_flops = 0;
  // partitioned low-rank powers: records (compute type) per operator and
  // stage, their rank table, FP64 scratch of the compression, compression
  // jobs, stage units per class, the stages each class may run in PLR form
  // and (once the ranks are read back at prepare) those it does
  int plr_digits = 0;
  Region r_plr, r_plr_rank, r_plr_q;
  std::vector<PlrJob> plr_jobs;
  std::vector<int64_t> plr_rec_off;
  std::vector<int32_t> plr_rank_off;
  std::vector<PlrUnit> plr_units;
  int plr_start[4] = {0, 0, 0, 0}, plr_count[4] = {0, 0, 0, 0};
  std::vector<int> plr_ok[4], plr_use[4];
  std::vector<int32_t> plr_ranks_host;
  int plr_max_s = 0, plr_stages = 0;
  double plr_flops = 0, plr_dense_flops = 0;
  size_t m_plr_jobs = 0, m_plr_recoff = 0, m_plr_rankoff = 0, m_plr_units = 0;
  // persistent launch
  std::vector<PItem> items;
  std::vector<int32_t> cnt_off, ntiles;
  int64_t n_counters = 0;
  int persistent_grid = 0;
  int32_t spin_limit = 0;  // bound of a persistent item's wait (0: the default)
  size_t m_items = 0, m_cntoff = 0, m_ntiles = 0, m_counters = 0;
  // persistent launch on the resident-power code (chain, resident and input-pass items)
  bool persist_res = false;
  std::vector<RItem> ritems;
  std::vector<int32_t> cnt_target;
  size_t m_ritems = 0, m_cnttarget = 0, persist_lds = 0;
  // backward
  int n_ckpt = 0, n_seg = 0, chunk_rows = 256;
  int64_t sum_x = 0;  // elements of one state buffer (all sequences)
  Region r_ckpt, r_seg, r_xfinal, r_gfirst, r_part, r_g;
  std::vector<RedChunk> chunks;
  int class_chunk_start[4] = {0, 0, 0, 0}, class_chunk_count[4] = {0, 0, 0, 0};
  int64_t class_part_off[4] = {0, 0, 0, 0};
  int class_op_start[4] = {0, 0, 0, 0}, class_op_count[4] = {0, 0, 0, 0};
  int class_set_start[4] = {0, 0, 0, 0}, class_set_count[4] = {0, 0, 0, 0};
  int class_max_p[4] = {0, 0, 0, 0}, class_max_q[4] = {0, 0, 0, 0};
  std::vector<SumJob> sj_dp, sj_dbb, sj_dc, sj_dd;  // grouped by class
  std::vector<int32_t> set_ops;                      // operators ordered by set
  std::vector<ScatterJob> scat;                      // one per parameter set
  std::vector<GemmJob> bjobs;                        // FP64 jobs of the backward
  std::vector<std::pair<int, int>> bgroups, bdims;   // (start, count), (max M, max N)
  std::vector<int> bkind;                            // 0: GEMM, 1: axpy
  size_t m_chunks = 0, m_sj = 0, m_set_ops = 0, m_scat = 0, m_bjobs = 0;
  size_t grad_numel = 0;

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
    if (d.N < -30 || d.N > 62)
      return fail(SSM_E_INVALID, "seq %d: N=%d outside -30..62 (negative: automatic)", i, d.N);
    if (d.L < 1 || d.L > ((int64_t)1 << 31) - 1)
      return fail(SSM_E_INVALID, "seq %d: L=%lld outside 1..2^31-1", i, (long long)d.L);
    if (d.param_set < 0) return fail(SSM_E_INVALID, "seq %d: negative param_set", i);
    if (d.reserved != 0) return fail(SSM_E_INVALID, "seq %d: reserved must be 0", i);
    if (d.u_offset < 0 || d.y_offset < 0)
      return fail(SSM_E_INVALID, "seq %d: negative offset", i);
  }
  return SSM_OK;
}

void plan_backward(ssm_plan_s& P);
void plan_backward_jobs(ssm_plan_s& P);
void plan_plr(ssm_plan_s& P);
void plr_select(ssm_plan_s& P);

// Automatic N (a sequence given N < 0, tolerance 10^N): the largest it can
// take is the smallest N whose window 2^(N+1) covers the sequence, where the
// cascade is exact (ceil(log2 L) - 1; 0 for L <= 2).
int auto_cap(int64_t L) {
  int n = 0;
  while (((int64_t)1 << (n + 1)) < L) ++n;
  return n;
}

// The descriptors with every automatic N at its cap; *any says whether one was.
std::vector<ssm_seq_desc> with_caps(const ssm_seq_desc* seqs, int32_t n_seq, bool* any) {
  std::vector<ssm_seq_desc> d(seqs, seqs + std::max(n_seq, 0));
  *any = false;
  for (ssm_seq_desc& x : d)
    if (x.N < 0) {
      *any = true;
      x.N = auto_cap(x.L);
    }
  return d;
}

// Builds sequences, operators, tiles, info and the workspace layout.
ssm_status build_plan(ssm_plan_s& P, const ssm_seq_desc* seqs, int32_t n_seq, ssm_disc disc,
                      ssm_dtype compute, int32_t with_backward, int32_t ckpt_every,
                      const ssm_tuning* tuning, bool norms_region = false) {
  ssm_status st = validate_seqs(seqs, n_seq);
  if (st != SSM_OK) return st;
  for (int i = 0; i < n_seq; ++i)
    if (seqs[i].N < 0) return fail(SSM_E_INVALID, "seq %d: automatic N not resolved", i);
  ssm_tuning tn{};
  if (tuning) tn = *tuning;
  if (tn.min_padded_m != 0 && tn.min_padded_m != 32 && tn.min_padded_m != 64 && tn.min_padded_m != 128 &&
      tn.min_padded_m != 256)
    return fail(SSM_E_INVALID, "min_padded_m = %d: supported 0, 32, 64, 128 or 256", tn.min_padded_m);
  P.min_mp = tn.min_padded_m > 0 ? tn.min_padded_m : 32;
  if (tn.plr_digits < 0 || tn.plr_digits > 15)
    return fail(SSM_E_INVALID, "plr_digits = %d: supported 0 (off) or 1..15", tn.plr_digits);
  if (tn.plr_digits > 0) {
    // the PLR stage runs FP32 or FP64 products, in the forward apply, per stage
    if (compute == SSM_BF16)
      return fail(SSM_E_UNSUPPORTED, "PLR powers: FP32 or FP64 compute (BF16 plans keep the fused dense passes)");
    if (with_backward) return fail(SSM_E_UNSUPPORTED, "PLR powers: forward only (with_backward is set)");
    if (tn.launch == SSM_LAUNCH_PERSISTENT)
      return fail(SSM_E_UNSUPPORTED, "PLR powers need per-stage launches (launch is persistent)");
    tn.launch = SSM_LAUNCH_PER_STAGE;
  }
  P.plr_digits = norms_region ? 0 : tn.plr_digits;
  if (tn.final_state < 0 || tn.final_state > 1)
    return fail(SSM_E_INVALID, "final_state = %d: supported 0 or 1", tn.final_state);
  if (tn.final_state) {
    // the final state is kept by the per-stage kernels' epilogues only: no
    // stage pairs, output fold or BF16 state, and per-stage launches
    if (tn.launch == SSM_LAUNCH_PERSISTENT)
      return fail(SSM_E_UNSUPPORTED, "final_state needs per-stage launches (launch is persistent)");
    tn.launch = SSM_LAUNCH_PER_STAGE;
    tn.pair_stages = 1;
    tn.fold_stages = -1;
    tn.state_bf16 = 0;
  }
  P.final_state = tn.final_state;
  if (tn.static_state < 0 || tn.static_state > 1)
    return fail(SSM_E_INVALID, "static_state = %d: supported 0 or 1", tn.static_state);
  if (tn.static_state && with_backward)
    return fail(SSM_E_UNSUPPORTED, "static_state: the backward needs the state buffers in the workspace");
  P.static_state = tn.static_state;
  if (tn.spin_limit < 0) return fail(SSM_E_INVALID, "spin_limit = %d: must be >= 0", tn.spin_limit);
  P.spin_limit = tn.spin_limit;
  if (tn.stage_kernel < SSM_STAGE_AUTO || tn.stage_kernel > SSM_STAGE_CHAIN)
    return fail(SSM_E_INVALID, "unknown stage kernel %d", tn.stage_kernel);
  if ((tn.stage_kernel == SSM_STAGE_RESIDENT || tn.stage_kernel == SSM_STAGE_CHAIN) &&
      compute == SSM_F64)
    return fail(SSM_E_UNSUPPORTED, "the resident and chain stage kernels take BF16 or FP32 operands");
  if (tn.chain_blocks < 0 || tn.chain_blocks > 64)
    return fail(SSM_E_INVALID, "chain_blocks = %d: supported 0 (automatic) or 1..64", tn.chain_blocks);
  if (tn.pair_stages < 0 || tn.pair_stages > 1)
    return fail(SSM_E_INVALID, "pair_stages = %d: supported 0 (automatic) or 1 (off)", tn.pair_stages);
  if (tn.pair_blocks != 0 && (tn.pair_blocks < 4 || tn.pair_blocks > 256))
    return fail(SSM_E_INVALID, "pair_blocks = %d: supported 0 (automatic) or 4..256", tn.pair_blocks);
  if (tn.input_split < 0 || tn.input_split > 1)
    return fail(SSM_E_INVALID, "input_split = %d: supported 0 (automatic) or 1 (off)", tn.input_split);
  if (tn.fold_stages < -1 || tn.fold_stages == 1 || tn.fold_stages > 6)
    return fail(SSM_E_INVALID, "fold_stages = %d: supported 0 (automatic), -1 (off) or 2..6", tn.fold_stages);
  if (tn.state_bf16 < 0 || tn.state_bf16 > 1)
    return fail(SSM_E_INVALID, "state_bf16 = %d: supported 0 (FP32 state) or 1 (BF16 where supported)",
                tn.state_bf16);
  if (tn.stage_kernel == SSM_STAGE_TILED || compute == SSM_F64)
    P.stage_kernel = SSM_STAGE_TILED;
  else
    P.stage_kernel = tn.stage_kernel == SSM_STAGE_RESIDENT ? SSM_STAGE_RESIDENT : SSM_STAGE_CHAIN;
  if (tn.launch < SSM_LAUNCH_AUTO || tn.launch > SSM_LAUNCH_PERSISTENT)
    return fail(SSM_E_INVALID, "unknown launch mode %d", tn.launch);
  for (int c = 0; c < 4; ++c) {
    const int d = stage_bm(kClassMp[c], (int)compute);
    const int r = tn.tile_rows[c];
    if (r != 0 && r != d && r != d / 2)
      return fail(SSM_E_INVALID, "tile_rows[%d] = %d: supported %d or %d", c, r, d, d / 2);
    P.class_bm[c] = r ? r : d;
  }
  if (disc != SSM_DISC_TRAPEZOID && disc != SSM_DISC_GIVEN && disc != SSM_DISC_ZOH)
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
    const bool uses_delta = disc == SSM_DISC_TRAPEZOID || disc == SSM_DISC_ZOH;
    if (uses_delta && !(d.delta > 0.0 && std::isfinite(d.delta)))
      return fail(SSM_E_INVALID, "seq %d: delta must be positive and finite", i);
    uint64_t dbits = 0;
    if (uses_delta) std::memcpy(&dbits, &d.delta, 8);
    auto key = std::make_pair(d.param_set, dbits);
    int op;
    auto it = key2op.find(key);
    const int lst = last_stage(d.N, d.L);
    if (it == key2op.end()) {
      op = (int)P.ops.size();
      key2op[key] = op;
      OpDev o{};
      o.m = d.m;
      o.mp = std::max(pad_m(d.m), P.min_mp);
      o.p = d.p;
      o.q = d.q;
      o.set = d.param_set;
      o.delta = uses_delta ? d.delta : 0.0;
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
    const int bm = P.class_bm[c];
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

  // row ranges of the resident-power kernel (about 512 per class)
  P.ranges.clear();
  P.chain_units.clear();
  for (int c = 0; c < 4; ++c) {
    std::vector<int> ids;
    int64_t rows = 0;
    for (int i = 0; i < n_seq; ++i)
      if (P.ops[P.seqs[i].op].mp == kClassMp[c]) {
        ids.push_back(i);
        rows += P.seqs[i].L;
      }
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int a, int b) { return P.seqs[a].last > P.seqs[b].last; });
    const int64_t R = std::max<int64_t>(128, ((rows + 511) / 512 + 127) / 128 * 128);
    P.class_range_start[c] = (int)P.ranges.size();
    for (int i : ids)
      for (int64_t r0 = 0; r0 < P.seqs[i].L; r0 += R)
        P.ranges.push_back(ResRange{i, (int32_t)r0, (int32_t)std::min<int64_t>(R, P.seqs[i].L - r0), 0});
    P.class_range_count[c] = (int)P.ranges.size() - P.class_range_start[c];
    const int ml = P.class_max_last[c];
    P.class_range_active[c].assign(ml + 1, 0);
    P.class_final[c].assign(ml + 1, 0);
    for (int kk = 0; kk <= ml; ++kk) {
      int cnt = 0;
      for (int r = P.class_range_start[c]; r < (int)P.ranges.size(); ++r)
        if (P.seqs[P.ranges[r].seq].last >= kk) ++cnt;
      P.class_range_active[c][kk] = cnt;
    }
    for (int i : ids) P.class_final[c][P.seqs[i].last] += 1;

    // chain-kernel units for the stages with 2^k >= 16: per sequence (longest
    // running first) its segments of T blocks, eight per workgroup
    P.chain_start[c].assign(ml + 1, 0);
    P.chain_count[c].assign(ml + 1, 0);
    P.chain_T[c].assign(ml + 1, 0);
    if (P.stage_kernel != SSM_STAGE_CHAIN || !chain_supported(kClassMp[c], (int)compute)) continue;
    // the chain kernel addresses a sequence's state with 32-bit byte offsets
    bool fits = true;
    for (int i : ids) fits = fits && P.seqs[i].L * (int64_t)kClassMp[c] * 4 <= ((int64_t)1 << 31);
    if (!fits) continue;
    for (int kk = 4; kk <= ml; ++kk) {
      const int64_t sh = (int64_t)1 << kk;
      // blocks of 16 rows, numbered column by column (column = rows equal mod 2^k
      // in 16-row groups); each wave takes T consecutive blocks
      int64_t blocks = 0;
      for (int i : ids)
        if (P.seqs[i].last >= kk) blocks += (sh / 16) * ((P.seqs[i].L + sh - 1) / sh);
      const int T = tn.chain_blocks > 0 ? tn.chain_blocks
                                        : (int)std::min<int64_t>(8, std::max<int64_t>(1, blocks / 2048));
      P.chain_T[c][kk] = T;
      P.chain_start[c][kk] = (int)P.chain_units.size();
      for (int i : ids) {
        if (P.seqs[i].last < kk) continue;
        const int64_t nflat = (sh / 16) * ((P.seqs[i].L + sh - 1) / sh);
        const int64_t nseg = (nflat + T - 1) / T;
        for (int64_t g0 = 0; g0 < nseg; g0 += 8)
          P.chain_units.push_back(ChainUnit{i, (int32_t)g0, T, 0});
      }
      P.chain_count[c][kk] = (int)P.chain_units.size() - P.chain_start[c][kk];
    }
  }

  // launch mode: persistent for ragged batches unless asked otherwise
  {
    int classes = 0, lmin = 1 << 30, lmax = -1;
    for (int c = 0; c < 4; ++c) classes += P.class_tile_count[c] > 0;
    for (const SeqDev& sq : P.seqs) {
      lmin = std::min(lmin, sq.last);
      lmax = std::max(lmax, sq.last);
    }
    P.launch = tn.launch == SSM_LAUNCH_AUTO
                   ? ((classes > 1 || lmin != lmax) ? SSM_LAUNCH_PERSISTENT : SSM_LAUNCH_PER_STAGE)
                   : tn.launch;
  }
  // The persistent launch runs the resident-power code when every operator
  // allows it: chain-capable sizes, at least one stage foldable into the input
  // pass (2p <= padded m) and sequences within 32-bit chain offsets.
  P.persist_res = false;
  if (P.launch == SSM_LAUNCH_PERSISTENT && P.stage_kernel != SSM_STAGE_TILED &&
      tn.input_stages >= 0) {
    bool ok = true;
    for (const OpDev& o : P.ops)
      ok = ok && chain_supported(o.mp, (int)compute) && !res_splits_rows(o.mp, (int)compute) &&
           2 * o.p <= o.mp;
    for (const SeqDev& sq : P.seqs)
      ok = ok && sq.L * (int64_t)P.ops[sq.op].mp * 4 <= ((int64_t)1 << 31);
    P.persist_res = ok;
  }
  // leading stages folded into the input pass (resident kernel, per-stage
  // launches or the resident persistent launch)
  P.max_kry = 0;
  // The split input pass (K_j rows in registers) folds stages while
  // 2^j p <= 2 mp, for operators whose sequences all run stages past j and
  // whole classes of such operators sharing p and j (per-stage launches of the
  // chain kernels); the resident input pass folds while 2^j p <= mp.
  const int nops = (int)P.ops.size();
  std::vector<int> jres(nops, 0), jsplit(nops, 0);
  bool class_split[4] = {true, true, true, true}, class_has[4] = {false, false, false, false};
  for (int oi = 0; oi < nops; ++oi) {
    const OpDev& o = P.ops[oi];
    int j = 0, jw = 0;
    while (((int64_t)o.p << (j + 1)) <= o.mp && j + 1 <= o.N + 1) ++j;
    while (((int64_t)o.p << (jw + 1)) <= 2 * (int64_t)o.mp && jw + 1 <= o.N + 1) ++jw;
    if (tn.input_stages > 0) {
      j = std::min(j, tn.input_stages);
      jw = std::min(jw, tn.input_stages);
    }
    jres[oi] = j;
    bool split = P.launch == SSM_LAUNCH_PER_STAGE && P.stage_kernel == SSM_STAGE_CHAIN &&
                 tn.input_split != 1 && tn.input_stages >= 0 && jw >= 2 &&
                 input_split_supported(o.mp, (int)compute, o.p, o.p << jw);
    for (const SeqDev& sq : P.seqs)
      if (sq.op == oi) split = split && jw <= sq.last;
    jsplit[oi] = split ? jw : 0;
    const int c = class_of(o.mp);
    if (!class_has[c]) {
      P.class_input_p[c] = o.p;
      P.class_input_kdim[c] = o.p << jw;
    }
    class_has[c] = true;
    class_split[c] = class_split[c] && split && o.p == P.class_input_p[c] &&
                     (o.p << jw) == P.class_input_kdim[c];
  }
  for (int oi = 0; oi < nops; ++oi) {
    OpDev& o = P.ops[oi];
    o.kry = 0;
    o.kdim = 0;
    o.kst = o.mp;
    o.ksplit = 0;
    o.kw = o.kc = -1;
    o.cpw = o.cpc = -1;
    o.cpl = -1;
    if (tn.input_stages < 0 || !(P.launch == SSM_LAUNCH_PER_STAGE || P.persist_res) ||
        P.stage_kernel == SSM_STAGE_TILED || !res_supported(o.mp, P.compute))
      continue;
    const int c = class_of(o.mp);
    if (class_has[c] && class_split[c]) {
      o.kry = jsplit[oi];
      o.kdim = o.p << o.kry;
      o.kst = std::max(o.mp, o.kdim);
      o.ksplit = 1;
    } else if (jres[oi] >= (P.persist_res ? 1 : 2)) {  // the persistent items start with an input pass
      o.kry = jres[oi];
      o.kdim = o.p << o.kry;
    }
  }
  for (int c = 0; c < 4; ++c) {
    P.class_min_kry[c] = 1 << 30;
    P.class_all_kry[c] = 1;
  }
  for (SeqDev& sq : P.seqs) {
    const OpDev& o = P.ops[sq.op];
    int kr = std::min(o.kry, sq.last + 1);
    if (kr == sq.last + 1 && res_splits_rows(o.mp, P.compute)) kr = sq.last;
    if (kr < (P.persist_res ? 1 : 2)) kr = 0;
    sq.kry = kr;
    P.max_kry = std::max(P.max_kry, kr);
    const int c = class_of(o.mp);
    P.class_min_kry[c] = std::min(P.class_min_kry[c], kr);
    if (kr == 0) P.class_all_kry[c] = 0;
  }
  for (int c = 0; c < 4; ++c)
    if (P.class_min_kry[c] == (1 << 30)) P.class_min_kry[c] = 0;

  // split input pass units: row ranges of R rows (R p elements of input
  // staged per workgroup, about 256 ranges per class), longest sequences first
  P.input_units.clear();
  for (int c = 0; c < 4; ++c) {
    P.class_input_start[c] = (int)P.input_units.size();
    P.class_input_count[c] = 0;
    P.class_input_lds[c] = 0;
    if (!(class_has[c] && class_split[c])) continue;
    std::vector<int> ids;
    int64_t rows = 0;
    int maxp = 4, maxlag = 0;
    for (int i = 0; i < n_seq; ++i)
      if (P.ops[P.seqs[i].op].mp == kClassMp[c]) {
        ids.push_back(i);
        rows += P.seqs[i].L;
        maxp = std::max(maxp, P.seqs[i].p);
        maxlag = std::max(maxlag, (1 << P.seqs[i].kry) - 1);
      }
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
    int64_t R = std::min<int64_t>(1024, std::max<int64_t>(256, (rows / 256 + 15) / 16 * 16));
    while (R > 16 && (R + maxlag) * maxp * 2 > 65536) R -= 16;
    for (int i : ids)
      for (int64_t r0 = 0; r0 < P.seqs[i].L; r0 += R)
        P.input_units.push_back(ResRange{i, (int32_t)r0, (int32_t)std::min<int64_t>(R, P.seqs[i].L - r0), 0});
    P.class_input_count[c] = (int)P.input_units.size() - P.class_input_start[c];
    P.class_input_lds[c] = (size_t)(R + maxlag) * maxp * 2;
  }

  // Output pass with the last s stages folded in (forward apply, per-stage
  // launches of the chain kernels, BF16 at padded m 128 and 256): for classes
  // whose sequences all end at the same stage and share the folded input
  // stages, q <= 16 and p <= 64; s as large as the LDS holds the 2^s G_j and
  // such that the stages between the input pass and the fold pair up.
  P.seq_fold_s.assign(n_seq, 0);
  P.seq_fold_k0.assign(n_seq, 0);
  P.mixed_folds.clear();
  for (int c = 0; c < 4; ++c) {
    P.fold_s[c] = P.fold_k0[c] = 0;
    P.fold_wide[c] = false;
    P.fold_mixed[c] = false;
    if (P.class_max_last[c] < 0 || tn.fold_stages == -1 || P.launch != SSM_LAUNCH_PER_STAGE ||
        P.stage_kernel != SSM_STAGE_CHAIN || !fold_supported(kClassMp[c], (int)compute, 2))
      continue;
    int min_last = 1 << 30, max_last = -1, kmin = 1 << 30, kmax = -1, max_q = 1, max_p = 1;
    bool ok = true;
    for (const SeqDev& sq : P.seqs)
      if (P.ops[sq.op].mp == kClassMp[c]) {
        min_last = std::min(min_last, sq.last);
        max_last = std::max(max_last, sq.last);
        kmin = std::min(kmin, sq.kry);
        kmax = std::max(kmax, sq.kry);
        max_q = std::max(max_q, sq.q);
        max_p = std::max(max_p, sq.p);
        ok = ok && sq.q <= 16 && sq.p <= 64 && sq.L * (int64_t)kClassMp[c] * 4 <= ((int64_t)1 << 31);
      }
    if (ok && min_last != max_last && kmin == kmax && kmin >= 4 && tn.pair_stages != 1 &&
        pair_supported(kClassMp[c], (int)compute)) {
      // ragged class: every sequence's own fold depth s_i (the largest the
      // kernels take with last - s_i + 1 - kry even, so that stage pairs from
      // the input pass end right before it); operators shared by sequences
      // that would fold differently keep the class on single stages
      const int mp = kClassMp[c];
      const int cap = tn.fold_stages > 0 ? tn.fold_stages : 6;
      std::map<int, std::pair<int, int>> op_fold;
      bool all = true;
      std::vector<std::pair<int, int>> pick(n_seq, {0, 0});
      for (int i = 0; i < n_seq && all; ++i) {
        const SeqDev& sq = P.seqs[i];
        if (P.ops[sq.op].mp != mp) continue;
        const int rem = sq.last - kmin + 1;
        int sf = 0;
        for (int t = std::min(rem, cap); t >= 2 && !sf; --t) {
          if ((rem - t) % 2) continue;
          if (t == 6 ? fold_wide_supported(mp, (int)compute, sq.q, sq.p) : t <= fold_max_stages(mp)) sf = t;
        }
        if (!sf) {
          all = false;
          break;
        }
        const std::pair<int, int> f{sf, sq.last - sf + 1};
        auto it = op_fold.find(sq.op);
        if (it != op_fold.end() && it->second != f) all = false;
        op_fold[sq.op] = f;
        pick[i] = f;
      }
      if (all) {
        P.fold_mixed[c] = true;
        for (int i = 0; i < n_seq; ++i)
          if (P.ops[P.seqs[i].op].mp == mp) {
            P.seq_fold_s[i] = pick[i].first;
            P.seq_fold_k0[i] = pick[i].second;
          }
      }
      continue;
    }
    if (!ok || min_last != max_last || kmin != kmax) continue;
    const bool wide_ok = fold_wide_supported(kClassMp[c], (int)compute, max_q, max_p);
    const int smax = std::min(wide_ok ? 6 : fold_max_stages(kClassMp[c]), tn.fold_stages > 0 ? tn.fold_stages : 99);
    for (int sf = smax; sf >= 2; --sf) {
      const int k0 = max_last - sf + 1, kp = std::max(4, kmin);
      if (k0 < 4 || k0 < kmin) continue;
      if (sf < 6 && sf > fold_max_stages(kClassMp[c])) continue;  // only the wide kernel folds six
      if (tn.pair_stages != 1 && pair_supported(kClassMp[c], (int)compute) && (k0 - kp) % 2 != 0) continue;
      P.fold_s[c] = sf;
      P.fold_k0[c] = k0;
      P.fold_wide[c] = sf == 6;
      break;
    }
  }

  // Stage pairs (forward apply, per-stage launches): stages k, k + 1 fused
  // where every sequence of the class runs both as lean stages, i.e. from the
  // largest folded stage count on and below the earliest last stage; the last
  // two stages fuse too (tail pair, which forms y) when every sequence of the
  // class ends at the same stage, q <= 16 and p <= 256. Units are segments of T blocks
  // in the numbering of stage k, longest sequences first (a tail segment's
  // inputs and D u are staged in LDS: T 16 (p + q) 4 bytes <= 64 KiB).
  P.pair_units.clear();
  for (int c = 0; c < 4; ++c) {
    const int ml = P.class_max_last[c];
    P.pair_start[c].assign(std::max(ml + 1, 0), 0);
    P.pair_count[c].assign(std::max(ml + 1, 0), 0);
    P.pair_tail[c].assign(std::max(ml + 1, 0), 0);
    P.pair_lds_bytes[c].assign(std::max(ml + 1, 0), 0);
    if (ml < 0 || tn.pair_stages == 1 || P.launch != SSM_LAUNCH_PER_STAGE ||
        P.stage_kernel != SSM_STAGE_CHAIN || !pair_supported(kClassMp[c], (int)compute))
      continue;
    std::vector<int> ids;
    int max_kry = 0, min_last = 1 << 30, max_last = -1, max_q = 1, max_p = 1;
    bool fits = true, small_io = true;
    for (int i = 0; i < n_seq; ++i)
      if (P.ops[P.seqs[i].op].mp == kClassMp[c]) {
        const SeqDev& sq = P.seqs[i];
        ids.push_back(i);
        max_kry = std::max(max_kry, sq.kry);
        min_last = std::min(min_last, sq.last);
        max_last = std::max(max_last, sq.last);
        max_q = std::max(max_q, sq.q);
        max_p = std::max(max_p, sq.p);
        fits = fits && sq.L * (int64_t)kClassMp[c] * 4 <= ((int64_t)1 << 31);
        small_io = small_io && sq.q <= 16 && sq.p <= 256;  // the tail's staged inputs fit in LDS
      }
    if (!fits) continue;
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
    // (with a fold, the pairs stop at its first stage and there is no tail
    // pair; a ragged class with per-sequence folds pairs each sequence up to
    // its own fold)
    int pair_end = P.fold_s[c] > 0 ? P.fold_k0[c] - 1 : min_last;
    if (P.fold_mixed[c]) {
      pair_end = 0;
      for (int i : ids) pair_end = std::max(pair_end, P.seq_fold_k0[i] - 1);
    }
    auto pairs_at = [&](int i, int kk) { return !P.fold_mixed[c] || kk + 2 <= P.seq_fold_k0[i]; };
    for (int kk = std::max(4, max_kry); kk + 1 <= pair_end; kk += 2) {
      const bool tail = P.fold_s[c] == 0 && !P.fold_mixed[c] && kk + 1 == min_last;
      if (tail && !(min_last == max_last && small_io)) break;
      const int64_t sh = (int64_t)1 << kk;
      int64_t blocks = 0;
      for (int i : ids)
        if (pairs_at(i, kk)) blocks += (sh / 16) * ((P.seqs[i].L + sh - 1) / sh);
      int T = tn.pair_blocks > 0 ? tn.pair_blocks
                                 : (int)std::min<int64_t>(64, std::max<int64_t>(8, blocks / 256));
      if (tail) T = std::max(1, std::min(T, 65536 / (64 * (max_p + max_q))));
      P.pair_start[c][kk] = (int)P.pair_units.size();
      for (int i : ids) {
        if (!pairs_at(i, kk)) continue;
        const int64_t nflat = (sh / 16) * ((P.seqs[i].L + sh - 1) / sh);
        for (int64_t f0 = 0; f0 < nflat; f0 += T)
          P.pair_units.push_back(PairUnit{i, (int32_t)f0, T, 0});
      }
      P.pair_count[c][kk] = (int)P.pair_units.size() - P.pair_start[c][kk];
      P.pair_tail[c][kk] = tail;
      P.pair_lds_bytes[c][kk] = pair_lds(kClassMp[c], tail, T, max_p, max_q);
      if (tail)  // the tail pair forms C P_{k+1} y_{l-2^{k+1}} with C P_{k+1} precomputed
        for (OpDev& o : P.ops)
          if (class_of(o.mp) == c) o.cpl = kk + 1;
    }
  }

  // fold operators, units (four columns of stage k0 per workgroup, longest
  // sequences first) and LDS
  P.fold_units.clear();
  for (OpDev& o : P.ops) {
    o.fold_s = 0;
    o.fold_k0 = 0;
    o.fold_paired = 0;
  }
  for (int c = 0; c < 4; ++c) {
    P.fold_start[c] = (int)P.fold_units.size();
    P.fold_count[c] = 0;
    P.fold_lds_bytes[c] = 0;
    if (P.fold_mixed[c]) {
      // one launch per (kernel, depth, state buffer of the fold's input):
      // after the input pass (its output in buffer kry mod 2) each pair
      // moves a sequence to the other buffer, (k0 - kry) / 2 pairs in all
      std::map<std::tuple<int, int, int>, std::vector<int>> groups;
      for (int i = 0; i < n_seq; ++i) {
        const SeqDev& sq = P.seqs[i];
        if (class_of(P.ops[sq.op].mp) != c) continue;
        const int sf = P.seq_fold_s[i], k0 = P.seq_fold_k0[i];
        const int buf = (sq.kry & 1) ^ (((k0 - sq.kry) / 2) & 1);
        groups[std::make_tuple(sf == 6 ? 1 : 0, sf, buf)].push_back(i);
        OpDev& o = P.ops[sq.op];
        o.fold_s = sf;
        o.fold_k0 = k0;
        o.fold_paired = sf == 6 ? 1 : 0;
      }
      for (auto& g : groups) {
        std::vector<int>& ids = g.second;
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
        ssm_plan_s::FoldLaunch fl{};
        fl.c = c;
        fl.wide = std::get<0>(g.first);
        fl.s = std::get<1>(g.first);
        fl.buf = std::get<2>(g.first);
        fl.start = (int)P.fold_units.size();
        fl.max_p = 1;
        fl.q4 = true;
        int max_q = 1;
        for (int i : ids) {
          const SeqDev& sq = P.seqs[i];
          fl.max_p = std::max(fl.max_p, sq.p);
          max_q = std::max(max_q, sq.q);
          fl.q4 = fl.q4 && sq.q % 4 == 0 && sq.y_off % 4 == 0;
          const int ncol = (1 << P.seq_fold_k0[i]) / 16;
          for (int c0 = 0; c0 < ncol; c0 += fl.wide ? 1 : 4)
            P.fold_units.push_back(FoldUnit{i, c0, fl.wide ? 1 : std::min(4, ncol - c0), 0});
        }
        fl.count = (int)P.fold_units.size() - fl.start;
        fl.lds = fl.wide ? fold_wide_lds() : fold_lds(kClassMp[c], fl.s, fl.max_p, max_q);
        P.mixed_folds.push_back(fl);
      }
      continue;
    }
    if (P.fold_s[c] == 0) continue;
    std::vector<int> ids;
    int max_p = 1, max_q = 1;
    bool q4 = true;
    for (int i = 0; i < n_seq; ++i)
      if (P.ops[P.seqs[i].op].mp == kClassMp[c]) {
        ids.push_back(i);
        max_p = std::max(max_p, P.seqs[i].p);
        max_q = std::max(max_q, P.seqs[i].q);
        q4 = q4 && P.seqs[i].q % 4 == 0 && P.seqs[i].y_off % 4 == 0;
      }
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
    const int ncol = (1 << P.fold_k0[c]) / 16;
    if (P.fold_wide[c]) {
      // one column per workgroup: its eight waves split the 64 lags
      for (int i : ids)
        for (int c0 = 0; c0 < ncol; ++c0) P.fold_units.push_back(FoldUnit{i, c0, 1, 0});
      P.fold_lds_bytes[c] = fold_wide_lds();
    } else {
      for (int i : ids)
        for (int c0 = 0; c0 < ncol; c0 += 4)
          P.fold_units.push_back(FoldUnit{i, c0, std::min(4, ncol - c0), 0});
      P.fold_lds_bytes[c] = fold_lds(kClassMp[c], P.fold_s[c], max_p, max_q);
    }
    P.fold_count[c] = (int)P.fold_units.size() - P.fold_start[c];
    P.fold_max_p[c] = max_p;
    P.fold_q4[c] = q4;
    for (OpDev& o : P.ops)
      if (class_of(o.mp) == c) {
        o.fold_s = P.fold_s[c];
        o.fold_k0 = P.fold_k0[c];
        o.fold_paired = P.fold_wide[c] ? 1 : 0;
      }
  }

  // BF16 state between the passes of the forward apply: only where every pass
  // of every class is the split input pass, a stage pair, or the output fold
  // after them, and the last pass forms y (the only kernels that read and
  // write it)
  P.state_bf16 = 0;
  if (tn.state_bf16 == 1) {
    bool ok = true, any = false;
    for (int c = 0; c < 4 && ok; ++c) {
      if (P.class_max_last[c] < 0) continue;
      any = true;
      ok = P.class_input_count[c] > 0;
      if (P.fold_mixed[c]) continue;  // the split input pass, pairs and every sequence's fold
      int kk = P.class_min_kry[c];
      bool tail = false;
      while (ok && kk <= P.class_max_last[c]) {
        if (P.fold_s[c] > 0 && kk == P.fold_k0[c]) {
          tail = true;
          break;
        }
        ok = kk < (int)P.pair_count[c].size() && P.pair_count[c][kk] > 0;
        if (ok && P.pair_tail[c][kk]) {
          tail = kk + 1 == P.class_max_last[c];
          break;
        }
        kk += 2;
      }
      ok = ok && tail;
    }
    P.state_bf16 = ok && any;
  }

  plan_plr(P);

  // persistent work items, level by level (projection = level -1), longer
  // sequences first inside a level; default tile heights
  P.items.clear();
  P.ritems.clear();
  P.cnt_target.clear();
  P.cnt_off.assign(n_seq, 0);
  P.ntiles.assign(n_seq, 0);
  if (P.launch == SSM_LAUNCH_PERSISTENT && P.persist_res) {
    // levels kry - 1 (input pass) .. last per sequence, one counter each
    std::vector<int> order(n_seq);
    for (int i = 0; i < n_seq; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
    int64_t cnt = 1;  // counter 0 hands out tickets
    int maxl = 0;
    for (int i = 0; i < n_seq; ++i) {
      P.cnt_off[i] = (int32_t)cnt;
      cnt += P.seqs[i].last - P.seqs[i].kry + 2;
      maxl = std::max(maxl, P.seqs[i].last);
    }
    P.n_counters = cnt;
    P.cnt_target.assign((size_t)cnt, 0);
    const int64_t R = 1024;  // rows per input-pass or resident-stage item
    for (int lev = -1; lev <= maxl; ++lev) {
      int64_t blocks = 0;  // chain blocks at this level, for the segment length
      if (lev >= 4)
        for (int i = 0; i < n_seq; ++i) {
          const SeqDev& sq = P.seqs[i];
          if (lev >= sq.kry && lev <= sq.last)
            blocks += ((int64_t)1 << (lev - 4)) * ((sq.L + ((int64_t)1 << lev) - 1) >> lev);
        }
      // longer segments than the per-stage launch (fewer items, each paying one
      // power load and one acquire/release) while a level keeps several items
      // per compute unit
      const int T = tn.chain_blocks > 0 ? tn.chain_blocks
                                        : (int)std::min<int64_t>(32, std::max<int64_t>(1, blocks / 8192));
      for (int i : order) {
        const SeqDev& sq = P.seqs[i];
        if (lev < sq.kry - 1 || lev > sq.last) continue;
        int32_t& target = P.cnt_target[P.cnt_off[i] + (lev - (sq.kry - 1))];
        if (lev == sq.kry - 1) {
          for (int64_t r0 = 0; r0 < sq.L; r0 += R) {
            P.ritems.push_back(RItem{i, -1, RI_INPUT, (int32_t)r0,
                                     (int32_t)std::min<int64_t>(R, sq.L - r0), lev, 0, 0});
            ++target;
          }
        } else if (lev >= 4) {
          const int64_t sh = (int64_t)1 << lev;
          const int64_t nflat = (sh / 16) * ((sq.L + sh - 1) / sh);
          const int64_t nseg = (nflat + T - 1) / T;
          const int per_unit = 8 * chain_segments_persist(P.ops[sq.op].mp, (int)compute, lev == sq.last);
          for (int64_t g0 = 0; g0 < nseg; g0 += per_unit) {
            P.ritems.push_back(RItem{i, lev, RI_CHAIN, (int32_t)g0, T, lev, lev == sq.last ? 1 : 0, 0});
            ++target;
          }
        } else {
          for (int64_t r0 = 0; r0 < sq.L; r0 += R) {
            P.ritems.push_back(RItem{i, lev, RI_RES, (int32_t)r0,
                                     (int32_t)std::min<int64_t>(R, sq.L - r0), lev, 0, 0});
            ++target;
          }
        }
      }
    }
    int max_mp = 32;
    for (const OpDev& o : P.ops) max_mp = std::max(max_mp, o.mp);
    P.persist_lds = persist_res_lds((int)compute, max_mp);
  } else if (P.launch == SSM_LAUNCH_PERSISTENT) {
    std::vector<int> order(n_seq);
    for (int i = 0; i < n_seq; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
    int64_t cnt = 1;  // counter 0 hands out tickets
    int maxl = 0;
    for (int i = 0; i < n_seq; ++i) {
      const int mp = P.ops[P.seqs[i].op].mp;
      const int bm = stage_bm(mp, P.compute);
      P.ntiles[i] = (int32_t)((P.seqs[i].L + bm - 1) / bm);
      P.cnt_off[i] = (int32_t)cnt;
      cnt += P.seqs[i].last + 2;
      maxl = std::max(maxl, P.seqs[i].last);
    }
    P.n_counters = cnt;
    for (int lev = -1; lev <= maxl; ++lev) {
      for (int i : order) {
        const SeqDev& sq = P.seqs[i];
        if (lev > sq.last) continue;
        const int mp = P.ops[sq.op].mp;
        const int bm = stage_bm(mp, P.compute);
        for (int t = 0; t < P.ntiles[i]; ++t) P.items.push_back(PItem{i, lev, t * bm, mp});
      }
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
  // row once and write it once (state element size); the last stage writes y
  // (element of y) instead of the state. The shifted partner of a row is a
  // row of the same stage input, so it adds no compulsory traffic.
  const double xe = P.state_bf16 ? 2.0 : (double)P.x_elem(), ye = (double)P.x_elem();
  auto pair_at = [&](int c, int kk) {
    return kk < (int)P.pair_count[c].size() && P.pair_count[c][kk] > 0;
  };
  P.stage_launches = 0;
  P.pair_launches = 0;
  P.pair_bytes = P.pair_flops = 0;
  P.fold_launches = 0;
  P.fold_bytes = P.fold_flops = 0;
  for (int c = 0; c < 4; ++c)
    if (P.class_max_last[c] >= 0 && P.fold_mixed[c]) {  // pairs, then the grouped folds
      for (int kk = 0; kk <= P.class_max_last[c]; ++kk)
        if (pair_at(c, kk)) {
          ++P.stage_launches;
          ++P.pair_launches;
        }
      for (const auto& fl : P.mixed_folds)
        if (fl.c == c) {
          ++P.stage_launches;
          ++P.fold_launches;
        }
    } else if (P.class_max_last[c] >= 0) {
      P.stage_launches += std::max(0, P.class_max_last[c] + 1 - P.class_min_kry[c]);
      for (int kk = 0; kk <= P.class_max_last[c]; ++kk)
        if (pair_at(c, kk)) {
          --P.stage_launches;  // two stages, one launch
          ++P.pair_launches;
        }
      if (P.fold_s[c] > 0) {  // the folded stages, one launch
        P.stage_launches -= P.fold_s[c] - 1;
        ++P.fold_launches;
      }
    }
  P.stage_flops = 0;
  for (int i = 0; i < n_seq; ++i) {
    const SeqDev& s = P.seqs[i];
    const int m = P.ops[s.op].m;
    const int c = class_of(P.ops[s.op].mp);
    // stages run as stage contractions: after the input pass, before a fold
    const int fs = P.fold_mixed[c] ? P.seq_fold_s[i] : P.fold_s[c];
    const int fk0 = P.fold_mixed[c] ? P.seq_fold_k0[i] : P.fold_k0[c];
    const int kend = fs > 0 ? fk0 - 1 : s.last;
    for (int kk = s.kry; kk <= kend; ++kk) {
      const int64_t sh = (int64_t)1 << kk;
      if (sh < s.L) P.stage_flops += 2.0 * m * m * (double)(s.L - sh);
    }
    if (fs > 0) {
      // the fold reads every state row once and writes y; row l takes
      // min(2^s, l / 2^k0 + 1) products with the q x m G_j
      const double in_row = (double)m * xe, out_row = (double)s.q * ye;
      P.stage_bytes += s.L * (in_row + out_row);
      P.fold_bytes += s.L * (in_row + out_row);
      const int64_t band = (int64_t)1 << fk0;
      for (int64_t b = 0; b * band < s.L; ++b)
        P.fold_flops += 2.0 * s.q * m * (double)std::min<int64_t>((int64_t)1 << fs, b + 1) *
                        (double)std::min<int64_t>(band, s.L - b * band);
    }
    for (int kk = s.kry; kk <= kend; ++kk) {
      const int kl = pair_at(c, kk) ? kk + 1 : kk;  // the launch's last stage
      const double in_row = (double)m * xe;
      const double out_row = kl == s.last ? (double)s.q * ye : (double)m * xe;
      P.stage_bytes += s.L * (in_row + out_row);
      if (pair_at(c, kk)) {  // the pair's second stage moves no further rows
        P.pair_bytes += s.L * (in_row + out_row);
        for (int h = 0; h < 2; ++h) {
          const int64_t sh = (int64_t)1 << (kk + h);
          if (sh < s.L) P.pair_flops += 2.0 * m * m * (double)(s.L - sh);
        }
        ++kk;
      }
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
         n_bsc = 0, n_kw = 0, n_zoh = 0;
  for (OpDev& o : P.ops) {
    const size_t mm = (size_t)o.mp * o.mp;
    o.pw = (int64_t)n_pw;
    n_pw += (size_t)(o.N + 1) * mm;
    o.pc = (int64_t)n_pc;
    n_pc += (size_t)(o.N + 1) * mm;
    if (o.kry > 0) {
      o.kc = (int64_t)n_pc;
      n_pc += (size_t)o.mp * o.kst;
      o.kw = (int64_t)n_kw;
      n_kw += (size_t)o.mp * o.kst;
    }
    if (o.cpl >= 0) {
      o.cpc = (int64_t)n_pc;
      n_pc += (size_t)16 * o.mp;
      o.cpw = (int64_t)n_kw;
      n_kw += (size_t)16 * o.mp;
    }
    o.fold_gw = o.fold_gc = -1;
    if (o.fold_s > 0) {
      const size_t ng = ((size_t)16 << o.fold_s) * o.mp;
      o.fold_gc = (int64_t)n_pc;
      n_pc += ng;
      o.fold_gw = (int64_t)n_kw;
      n_kw += ng;
    }
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
    n_small = (n_small + 3) & ~(size_t)3;  // 16-byte aligned rows for vector loads
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
    o.zx = -1;
    o.zn = o.zsq = 0;
    if (disc == SSM_DISC_ZOH) {
      o.zn = o.m + o.p;
      o.zx = (int64_t)n_zoh;
      n_zoh += (P.with_backward ? 6 : 3) * (size_t)o.zn * o.zn;
      P.z_nid = std::max(P.z_nid, o.zn);
    }
  }
  if (disc == SSM_DISC_ZOH) {
    P.z_id = (int64_t)n_zoh;
    n_zoh += (size_t)P.z_nid * P.z_nid;
    P.z_norm = (int64_t)n_zoh;
    n_zoh += P.ops.size();
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
  // lower-triangular test per operator: int flags, then FP64 scales
  P.m_tri = off;
  off = align_up(off + 4 * P.ops.size());
  P.m_tri_scale = off;
  off = align_up(off + 8 * P.ops.size());
  // jobs: 2 per operator (discretization) + one per operator and squaring
  size_t n_jobs = 2 * P.ops.size();
  for (const OpDev& o : P.ops)
    n_jobs += (size_t)o.N + (o.kry > 0 ? 1 + o.kry : 0) + (o.cpl >= 0) + (o.fold_s > 0 ? 1 + o.fold_s : 0);
  // doubling GEMMs of the triangular inverse: 2 (mp / 2s) per level s
  if (disc == SSM_DISC_TRAPEZOID)
    for (const OpDev& o : P.ops)
      for (int sz = 32; sz < o.mp; sz *= 2) n_jobs += 2 * (o.mp / (2 * sz));
  P.m_jobs = off;
  off = align_up(off + sizeof(GemmJob) * std::max<size_t>(1, n_jobs));
  // exponential discretization: per operator the scaling, the first Taylor
  // term, two jobs per Taylor step, up to kZohMaxSq squarings and two copies
  P.z_cap = disc == SSM_DISC_ZOH ? P.ops.size() * (size_t)(4 + 2 * kZohTaylor + kZohMaxSq) : 0;
  P.m_zjobs = off;
  off = align_up(off + sizeof(GemmJob) * std::max<size_t>(1, P.z_cap));
  // its adjoint: per operator five set-up jobs, four per Taylor step, three
  // per squaring and two copies
  P.zb_cap = disc == SSM_DISC_ZOH && P.with_backward
                 ? P.ops.size() * (size_t)(7 + 4 * kZohTaylor + 3 * kZohMaxSq) : 0;
  P.m_zbjobs = off;
  off = align_up(off + sizeof(GemmJob) * std::max<size_t>(1, P.zb_cap));
  P.sum_x = xoff;
  P.m_ranges = off;
  off = align_up(off + sizeof(ResRange) * std::max<size_t>(1, P.ranges.size()));
  P.m_chain = off;
  off = align_up(off + sizeof(ChainUnit) * std::max<size_t>(1, P.chain_units.size()));
  P.m_pair = off;
  off = align_up(off + sizeof(PairUnit) * std::max<size_t>(1, P.pair_units.size()));
  P.m_input = off;
  off = align_up(off + sizeof(ResRange) * std::max<size_t>(1, P.input_units.size()));
  P.m_fold = off;
  off = align_up(off + sizeof(FoldUnit) * std::max<size_t>(1, P.fold_units.size()));
  P.m_plr_jobs = off;
  off = align_up(off + sizeof(PlrJob) * std::max<size_t>(1, P.plr_jobs.size()));
  P.m_plr_recoff = off;
  off = align_up(off + sizeof(int64_t) * std::max<size_t>(1, P.plr_rec_off.size()));
  P.m_plr_rankoff = off;
  off = align_up(off + sizeof(int32_t) * std::max<size_t>(1, P.plr_rank_off.size()));
  P.m_plr_units = off;
  off = align_up(off + sizeof(PlrUnit) * std::max<size_t>(1, P.plr_units.size()));
  if (P.launch == SSM_LAUNCH_PERSISTENT) {
    P.m_ritems = off;
    off = align_up(off + sizeof(RItem) * std::max<size_t>(1, P.ritems.size()));
    P.m_cnttarget = off;
    off = align_up(off + sizeof(int32_t) * std::max<size_t>(1, P.cnt_target.size()));
    P.m_items = off;
    off = align_up(off + sizeof(PItem) * std::max<size_t>(1, P.items.size()));
    P.m_cntoff = off;
    off = align_up(off + sizeof(int32_t) * std::max<size_t>(1, P.cnt_off.size()));
    P.m_ntiles = off;
    off = align_up(off + sizeof(int32_t) * std::max<size_t>(1, P.ntiles.size()));
    P.m_counters = off;
    off = align_up(off + sizeof(int32_t) * ((size_t)P.n_counters + 1));  // + the give-up flag
  }
  if (P.with_backward) {
    plan_backward(P);
    size_t n_bjobs = 0;
    for (int k = 0; k < P.max_N; ++k)
      for (const OpDev& o : P.ops)
        if (o.N > k) n_bjobs += 2;
    n_bjobs += (disc == SSM_DISC_TRAPEZOID ? 5 : 2) * P.ops.size();
    P.m_chunks = off;
    off = align_up(off + sizeof(RedChunk) * std::max<size_t>(1, P.chunks.size()));
    P.m_sj = off;
    off = align_up(off + sizeof(SumJob) * std::max<size_t>(
                             1, P.sj_dp.size() + P.sj_dbb.size() + P.sj_dc.size() + P.sj_dd.size()));
    P.m_set_ops = off;
    off = align_up(off + sizeof(int32_t) * std::max<size_t>(1, P.set_ops.size()));
    P.m_scat = off;
    off = align_up(off + sizeof(ScatterJob) * std::max<size_t>(1, P.scat.size()) + 4096);
    P.m_bjobs = off;
    off = align_up(off + sizeof(GemmJob) * std::max<size_t>(1, n_bjobs));
  }
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
  take(P.r_kw, n_kw * 8);
  take(P.r_small, n_small * P.x_elem());
  take(P.r_aug, n_aug * 8);
  take(P.r_nmat, n_nmat * 8);
  take(P.r_bsc, n_bsc * 8);
  take(P.r_zoh, n_zoh * 8);
  P.n_norms = 0;
  if (norms_region)
    for (const OpDev& o : P.ops) P.n_norms += o.N + 1;
  take(P.r_norms, (size_t)P.n_norms * 8);
  take(P.r_plr, P.r_plr.bytes);
  take(P.r_plr_rank, P.r_plr_rank.bytes);
  take(P.r_plr_q, P.r_plr_q.bytes);
  P.x_buf_bytes = (size_t)xoff * P.x_elem();
  take(P.r_x0, P.static_state ? 0 : P.x_buf_bytes);
  take(P.r_x1, P.static_state ? 0 : P.x_buf_bytes);
  if (P.with_backward) {
    const size_t xb = (size_t)xoff * P.x_elem();
    take(P.r_ckpt, xb * P.n_ckpt);
    take(P.r_seg, xb * P.n_seg);
    take(P.r_xfinal, xb);
    take(P.r_gfirst, xb);
    take(P.r_part, P.r_part.bytes);
    take(P.r_g, P.r_g.bytes);
  }
  P.ws_bytes = cur;
  return SSM_OK;
}


// Partitioned low-rank powers: the stages each padded-size class may run in
// PLR form (per-stage launches of the forward apply, padded m 64..256, at or
// after every folded input stage of the class, before its earliest last stage
// so that no sequence forms y there, outside stage pairs and the output fold,
// every sequence's L mp bytes below 2^31), the row units of those classes,
// the records and rank slots of every operator of padded size >= 64, and a
// compression job per off-diagonal block (plus one for the leaves) of every
// eligible stage.
void plan_plr(ssm_plan_s& P) {
  P.plr_jobs.clear();
  P.plr_units.clear();
  P.plr_rec_off.assign(P.ops.size(), -1);
  P.plr_rank_off.assign(P.ops.size(), -1);
  P.plr_max_s = 0;
  for (int c = 0; c < 4; ++c) {
    P.plr_ok[c].clear();
    P.plr_use[c].clear();
    P.plr_start[c] = P.plr_count[c] = 0;
  }
  if (P.plr_digits <= 0 || P.launch != SSM_LAUNCH_PER_STAGE) return;
  const int64_t es = (int64_t)P.x_elem();
  for (int c = 1; c < 4; ++c) {
    const int mp = kClassMp[c];
    if (P.class_max_last[c] < 0) continue;
    int kmax = 0, lmin = 1 << 30;
    bool fits = true;
    std::vector<int> ids;
    for (int i = 0; i < P.n_seq; ++i) {
      const SeqDev& sq = P.seqs[i];
      if (P.ops[sq.op].mp != mp) continue;
      ids.push_back(i);
      kmax = std::max(kmax, sq.kry);
      lmin = std::min(lmin, sq.last);
      fits = fits && sq.L * mp * es < ((int64_t)1 << 31);
    }
    if (!fits) continue;
    P.plr_ok[c].assign(P.class_max_last[c] + 1, 0);
    P.plr_use[c].assign(P.class_max_last[c] + 1, 0);
    bool any = false;
    for (int k = kmax; k < lmin; ++k) {
      const bool paired = (k < (int)P.pair_count[c].size() && P.pair_count[c][k] > 0) ||
                          (k > 0 && k - 1 < (int)P.pair_count[c].size() && P.pair_count[c][k - 1] > 0);
      const bool folded = P.fold_s[c] > 0 && k >= P.fold_k0[c];
      if (paired || folded) continue;
      P.plr_ok[c][k] = 1;
      any = true;
    }
    if (!any) continue;
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return P.seqs[a].L > P.seqs[b].L; });
    P.plr_start[c] = (int)P.plr_units.size();
    const int rows = plr_unit_rows(P.compute);
    for (int i : ids)
      for (int64_t r0 = 0; r0 < P.seqs[i].L; r0 += rows) P.plr_units.push_back(PlrUnit{i, (int32_t)r0});
    P.plr_count[c] = (int)P.plr_units.size() - P.plr_start[c];
  }
  int64_t rec = 0, rk = 0;
  for (size_t oi = 0; oi < P.ops.size(); ++oi) {
    const OpDev& o = P.ops[oi];
    const int c = class_of(o.mp);
    if (o.mp < 64 || P.plr_ok[c].empty()) continue;
    P.plr_rec_off[oi] = rec;
    P.plr_rank_off[oi] = (int32_t)rk;
    rec += (int64_t)(o.N + 1) * plr_rec_elems(o.mp);
    rk += (int64_t)(o.N + 1) * kPlrRankSlots;
    const int D = plr_levels(o.mp);
    for (int k = 0; k <= o.N && k < (int)P.plr_ok[c].size(); ++k) {
      if (!P.plr_ok[c][k]) continue;
      P.plr_jobs.push_back(PlrJob{(int32_t)oi, k, 0, 0, 0, {0, 0, 0}});
      for (int d = 1; d <= D; ++d)
        for (int g = 0; g < (1 << (d - 1)); ++g)
          for (int side = 0; side < 2; ++side) P.plr_jobs.push_back(PlrJob{(int32_t)oi, k, d, g, side, {0, 0, 0}});
      P.plr_max_s = std::max(P.plr_max_s, o.mp / 2);
    }
  }
  P.r_plr.bytes = (size_t)rec * (P.compute == DT_F64 ? 8 : 4);
  P.r_plr_rank.bytes = (size_t)rk * 4;
  P.r_plr_q.bytes = P.plr_jobs.size() * (size_t)kPlrRC * kPlrMaxS * 8;
  P.plr_ranks_host.assign((size_t)rk, 0);
}

// Matrix-core steps (16 x 16 x 4) per 16 rows of one stage of operator o in
// PLR form with the ranks found at prepare: phase A ceil(r / 16) s / 4 per
// block of rank r > 0, phase B 4 per leaf plus ceil(r / 4) for every level's
// block over the leaf; -1 if a rank exceeds the cap.
static int64_t plr_steps(const int32_t* rk, int mp) {
  const int D = plr_levels(mp), NL = mp / kPlrLeaf;
  int64_t steps = 0;
  for (int d = 1; d <= D; ++d)
    for (int g = 0; g < (1 << (d - 1)); ++g)
      for (int side = 0; side < 2; ++side) {
        const int r = rk[plr_rank_index(d, g, side)];
        if (r > kPlrRC) return -1;
        if (r > 0) steps += (int64_t)((r + 15) / 16) * ((mp >> d) / 4);
      }
  for (int f = 0; f < NL; ++f) {
    steps += 4;
    for (int d = 1; d <= D; ++d) {
      const int h = NL >> d, hi = f / h;
      const int r = rk[plr_rank_index(d, hi >> 1, (hi & 1) ? 0 : 1)];
      steps += (r + 3) / 4;
    }
  }
  return steps;
}

// per row flops of the PLR form as applied: 2 (16 mp + sum over blocks 2 r s)
static double plr_row_flops(const int32_t* rk, int mp) {
  const int D = plr_levels(mp);
  double f = 16.0 * mp;
  for (int d = 1; d <= D; ++d)
    for (int g = 0; g < (1 << (d - 1)); ++g)
      for (int side = 0; side < 2; ++side) f += 2.0 * rk[plr_rank_index(d, g, side)] * (mp >> d);
  return 2.0 * f;
}

// After the ranks are read back: a class runs stage k in PLR form if every
// operator of the class fits the rank cap there and needs at most half the
// matrix-core steps of the dense product (mp / 16 output blocks of mp / 4).
void plr_select(ssm_plan_s& P) {
  P.plr_stages = 0;
  P.plr_flops = P.plr_dense_flops = 0;
  for (int c = 1; c < 4; ++c) {
    const int mp = kClassMp[c];
    for (int k = 0; k < (int)P.plr_ok[c].size(); ++k) {
      P.plr_use[c][k] = 0;
      if (!P.plr_ok[c][k]) continue;
      bool ok = true;
      for (size_t oi = 0; oi < P.ops.size() && ok; ++oi) {
        const OpDev& o = P.ops[oi];
        if (o.mp != mp || P.plr_rank_off[oi] < 0) continue;
        const int64_t st = plr_steps(P.plr_ranks_host.data() + P.plr_rank_off[oi] + k * kPlrRankSlots, mp);
        ok = st >= 0 && 2 * st <= (int64_t)(mp / 16) * (mp / 4);
      }
      if (!ok) continue;
      P.plr_use[c][k] = 1;
      ++P.plr_stages;
      for (const SeqDev& sq : P.seqs) {
        const OpDev& o = P.ops[sq.op];
        if (o.mp != mp) continue;
        const double rows = (double)std::max<int64_t>(0, sq.L - ((int64_t)1 << k));
        const int32_t* rk = P.plr_ranks_host.data() + P.plr_rank_off[sq.op] + k * kPlrRankSlots;
        P.plr_flops += rows * plr_row_flops(rk, mp);
        P.plr_dense_flops += rows * 2.0 * mp * mp;
      }
    }
  }
}

// Backward planning: checkpoint layout, reduction chunks, sum / GEMM /
// scatter job lists and the FP64 gradient workspace. Offsets of the
// workspace regions are assigned by the caller.
void plan_backward(ssm_plan_s& P) {
  const int c = P.ckpt_every;
  P.n_ckpt = (P.max_last + 1) / c + 1;  // inputs of stages 0, c, 2c, ... and possibly K
  P.n_seg = c - 1;
  // reduction chunks: bounded count
  int64_t rows = 0;
  for (const SeqDev& s : P.seqs) rows += s.L;
  P.chunk_rows = 256 * (int)std::max<int64_t>(1, (rows + 256 * 4096 - 1) / (256 * 4096));
  // operators ordered by set
  P.set_ops.clear();
  std::vector<std::vector<int>> ops_of_set(P.n_sets), seqs_of_op(P.n_ops);
  for (int o = 0; o < P.n_ops; ++o) ops_of_set[P.ops[o].set].push_back(o);
  for (int i = 0; i < P.n_seq; ++i) seqs_of_op[P.seqs[i].op].push_back(i);
  std::vector<int> set_op_first(P.n_sets, 0);
  for (int st = 0; st < P.n_sets; ++st) {
    set_op_first[st] = (int)P.set_ops.size();
    for (int o : ops_of_set[st]) P.set_ops.push_back(o);
  }
  // FP64 gradient workspace
  int64_t g = 0;
  for (OpDev& o : P.ops) {
    const int64_t mm = (int64_t)o.mp * o.mp;
    o.g_dp = g;
    g += (int64_t)(o.N + 1) * mm;
    o.g_dbb = g;
    g += (int64_t)o.mp * o.p;
    o.g_s = g;
    g += mm;
    o.g_da = g;
    g += mm;
    o.g_db = g;
    g += (int64_t)o.mp * o.p;
  }
  std::vector<int64_t> set_dc(P.n_sets, -1), set_dd(P.n_sets, -1);
  for (int st = 0; st < P.n_sets; ++st) {
    if (ops_of_set[st].empty()) continue;
    const OpDev& o = P.ops[ops_of_set[st][0]];
    set_dc[st] = g;
    g += (int64_t)o.q * o.mp;
    set_dd[st] = g;
    g += (int64_t)o.q * o.p;
  }
  P.r_g.bytes = (size_t)g * 8;
  // chunks and sum jobs, grouped by size class, then set, operator, sequence
  P.chunks.clear();
  P.sj_dp.clear();
  P.sj_dbb.clear();
  P.sj_dc.clear();
  P.sj_dd.clear();
  int64_t part = 0;
  for (int cl = 0; cl < 4; ++cl) {
    const int mp = kClassMp[cl];
    const int64_t mm = (int64_t)mp * mp;
    P.class_chunk_start[cl] = (int)P.chunks.size();
    P.class_op_start[cl] = (int)P.sj_dp.size();
    P.class_set_start[cl] = (int)P.sj_dc.size();
    P.class_max_p[cl] = P.class_max_q[cl] = 0;
    for (int st = 0; st < P.n_sets; ++st) {
      if (ops_of_set[st].empty() || P.ops[ops_of_set[st][0]].mp != mp) continue;
      const int set_first = (int)P.chunks.size() - P.class_chunk_start[cl];
      for (int o : ops_of_set[st]) {
        const OpDev& od = P.ops[o];
        const int op_first = (int)P.chunks.size() - P.class_chunk_start[cl];
        for (int sq : seqs_of_op[o]) {
          const int64_t L = P.seqs[sq].L;
          for (int64_t r0 = 0; r0 < L; r0 += P.chunk_rows) {
            RedChunk ch;
            ch.seq = sq;
            ch.row0 = (int32_t)r0;
            ch.nrows = (int32_t)std::min<int64_t>(P.chunk_rows, L - r0);
            ch.slot = (int32_t)P.chunks.size() - P.class_chunk_start[cl];
            P.chunks.push_back(ch);
          }
        }
        const int n = (int)P.chunks.size() - P.class_chunk_start[cl] - op_first;
        P.sj_dp.push_back(SumJob{op_first, n, (int32_t)mm, mm, od.g_dp, mm, od.N, 0});
        P.sj_dbb.push_back(SumJob{op_first, n, od.mp * od.p, mm, od.g_dbb, 0, 0, 0});
        P.class_max_p[cl] = std::max(P.class_max_p[cl], od.p);
        P.class_max_q[cl] = std::max(P.class_max_q[cl], od.q);
      }
      const OpDev& o0 = P.ops[ops_of_set[st][0]];
      const int n = (int)P.chunks.size() - P.class_chunk_start[cl] - set_first;
      P.sj_dc.push_back(SumJob{set_first, n, o0.q * o0.mp, mm, set_dc[st], 0, 0, 0});
      P.sj_dd.push_back(SumJob{set_first, n, o0.q * o0.p, mm, set_dd[st], 0, 0, 0});
    }
    P.class_chunk_count[cl] = (int)P.chunks.size() - P.class_chunk_start[cl];
    P.class_op_count[cl] = (int)P.sj_dp.size() - P.class_op_start[cl];
    P.class_set_count[cl] = (int)P.sj_dc.size() - P.class_set_start[cl];
    P.class_part_off[cl] = part;
    part += (int64_t)P.class_chunk_count[cl] * mm;
  }
  P.r_part.bytes = (size_t)part * P.x_elem();
  // scatter jobs (set sizes as seen from the sequences; prepare completes
  // unused sets from the parameter descriptors)
  P.scat.assign(P.n_sets, ScatterJob{});
  for (int st = 0; st < P.n_sets; ++st) {
    ScatterJob& j = P.scat[st];
    j.op_first = set_op_first[st];
    j.n_ops = (int)ops_of_set[st].size();
    j.m = std::max(0, P.set_m[st]);
    j.mp = j.m ? std::max(pad_m(j.m), P.min_mp) : 0;
    j.p = std::max(0, P.set_p[st]);
    j.q = std::max(0, P.set_q[st]);
    j.dC = set_dc[st];
    j.dD = set_dd[st];
    j.out = 0;
  }
}

// FP64 job lists of the backward (pointers into the workspace).
void plan_backward_jobs(ssm_plan_s& P) {
  double* pw = P.at<double>(P.r_pw);
  double* bbar = P.at<double>(P.r_bbar);
  double* minv = P.at<double>(P.r_minv);
  double* G = P.at<double>(P.r_g);
  P.bjobs.clear();
  P.bgroups.clear();
  P.bdims.clear();
  P.bkind.clear();
  auto close_group = [&](int start, int kind) {
    int mx = 0, mn = 0;
    for (size_t i = start; i < P.bjobs.size(); ++i) {
      mx = std::max(mx, P.bjobs[i].M);
      mn = std::max(mn, P.bjobs[i].N);
    }
    if ((int)P.bjobs.size() > start) {
      P.bgroups.push_back({start, (int)P.bjobs.size() - start});
      P.bdims.push_back({mx, mn});
      P.bkind.push_back(kind);
    }
  };
  // squaring adjoint: G_k += G_{k+1} P_k^T + P_k^T G_{k+1}, k = N-1..0
  for (int k = P.max_N - 1; k >= 0; --k) {
    for (int half = 0; half < 2; ++half) {
      int start = (int)P.bjobs.size();
      for (const OpDev& o : P.ops) {
        if (o.N <= k) continue;
        const int64_t mm = (int64_t)o.mp * o.mp;
        double* Gk = G + o.g_dp + k * mm;
        double* Gk1 = Gk + mm;
        double* Pk = pw + o.pw + k * mm;
        if (half == 0)
          P.bjobs.push_back(GemmJob{Gk1, Pk, Gk, o.mp, o.mp, o.mp, o.mp, o.mp, o.mp, 0, 1, 1.0, 1.0});
        else
          P.bjobs.push_back(GemmJob{Pk, Gk1, Gk, o.mp, o.mp, o.mp, o.mp, o.mp, o.mp, 1, 0, 1.0, 1.0});
      }
      close_group(start, 0);
    }
  }
  int start = (int)P.bjobs.size();
  if (P.disc == SSM_DISC_TRAPEZOID) {
    // S = G_Abar (I + Abar)^T + G_Bbar Bbar^T;  dA = delta/2 M^{-T} S;  dB = delta M^{-T} G_Bbar
    for (const OpDev& o : P.ops)
      P.bjobs.push_back(GemmJob{G + o.g_dp, pw + o.pw, G + o.g_s, o.mp, o.mp, o.mp, o.mp, o.mp,
                                o.mp, 0, 1, 1.0, 0.0});
    close_group(start, 0);
    start = (int)P.bjobs.size();
    for (const OpDev& o : P.ops)
      P.bjobs.push_back(GemmJob{G + o.g_dp, nullptr, G + o.g_s, o.mp, o.mp, 0, o.mp, 0, o.mp, 0, 0,
                                1.0, 1.0});
    close_group(start, 1);
    start = (int)P.bjobs.size();
    for (const OpDev& o : P.ops)
      P.bjobs.push_back(GemmJob{G + o.g_dbb, bbar + o.bbar, G + o.g_s, o.mp, o.mp, o.p, o.p, o.p,
                                o.mp, 0, 1, 1.0, 1.0});
    close_group(start, 0);
    start = (int)P.bjobs.size();
    for (const OpDev& o : P.ops) {
      P.bjobs.push_back(GemmJob{minv + o.minv, G + o.g_s, G + o.g_da, o.mp, o.mp, o.mp, o.mp, o.mp,
                                o.mp, 1, 0, 0.5 * o.delta, 0.0});
      P.bjobs.push_back(GemmJob{minv + o.minv, G + o.g_dbb, G + o.g_db, o.mp, o.p, o.mp, o.mp, o.p,
                                o.p, 1, 0, o.delta, 0.0});
    }
    close_group(start, 0);
  } else if (P.disc == SSM_DISC_GIVEN) {
    for (const OpDev& o : P.ops) {
      P.bjobs.push_back(GemmJob{G + o.g_dp, nullptr, G + o.g_da, o.mp, o.mp, 0, o.mp, 0, o.mp, 0, 0,
                                1.0, 0.0});
      P.bjobs.push_back(GemmJob{G + o.g_dbb, nullptr, G + o.g_db, o.mp, o.p, 0, o.p, 0, o.p, 0, 0,
                                1.0, 0.0});
    }
    close_group(start, 1);
  }
}

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
// uses it and it can apply this stage, the tiled one otherwise.
hipError_t launch_stage_any(const ssm_plan_s& P, int c, StageParams prm, hipStream_t stream) {
  const int mp = kClassMp[c];
  const int k = prm.k;
  if (k < (int)P.chain_count[c].size() && P.chain_count[c][k] > 0) {
    const ChainUnit* un = reinterpret_cast<const ChainUnit*>(P.ws + P.r_meta.off + P.m_chain) +
                          P.chain_start[c][k];
    const bool tail = prm.adjoint ? k == 0 : P.class_final[c][k] > 0;
    if (!(tail && res_splits_rows(mp, P.compute)))
      return launch_stage_chain(mp, P.compute, prm, un, P.chain_count[c][k], tail, stream);
  }
  const bool final_here = (prm.flags & SF_EPILOGUE) &&
                          (prm.adjoint ? k == 0 : (k < (int)P.class_final[c].size() &&
                                                   P.class_final[c][k] > 0));
  if (P.stage_kernel != SSM_STAGE_TILED && res_supported(mp, P.compute) &&
      !(final_here && res_splits_rows(mp, P.compute))) {
    const ResRange* rg = reinterpret_cast<const ResRange*>(P.ws + P.r_meta.off + P.m_ranges) +
                         P.class_range_start[c];
    return launch_stage_res(mp, P.compute, prm, rg, P.class_range_active[c][k], stream);
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
                            o.kst, 0, 0, 1.0, 0.0});
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
                          o.mp, 0, 0, 1.0, 0.0});
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
                            rows, o.mp, o.mp, o.mp, o.mp, o.mp, 0, 0, 1.0, 0.0});
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
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bail(hip_fail(e, "prepare synchronization"));
  if (status_h[0] != 0)
    return bail(fail(SSM_E_NUMERIC, "I - delta/2 A is singular to working precision"));
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
    prm.xfinal = xfinal;
    for (int k = 0; k <= ml; ++k) {
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
        prm.k = k;
        prm.xin = loc(k);
        prm.xout = loc(k + 1);
        prm.n_tiles = P.class_active[cl][k];
        TimedLaunch tl(P, stream, 0);
        e = launch_stage_any(P, cl, prm, stream);
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
  info->plr_stages = plan->plr_stages;
  info->plr_reserved = 0;
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
