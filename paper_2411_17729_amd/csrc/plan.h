// Host-side plan of the fast-cascade library: the plan structure, its
// workspace regions and the planning steps (validation, operators, work
// units of every kernel family, the workspace layout, the backward's jobs,
// the partitioned low-rank stages). Shared by the planning code (plan.cpp)
// and the entry points that launch a plan (api.cpp). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/ssm_cascade.h"
#include "plr.h"
#include "ssm_internal.h"

namespace ssmc {
namespace host {

// the message ssm_last_error returns (per thread)
extern thread_local std::string g_last_error;
// records the message and returns s
ssm_status fail(ssm_status s, const char* fmt, ...);
ssm_status hip_fail(hipError_t e, const char* what);

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

}  // namespace host
}  // namespace ssmc

// (internal header: the plan structure, at global scope as the ABI declares
// it, names the library's device descriptors and helpers directly)
using namespace ssmc;
using namespace ssmc::host;

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
  // (after prepare) every operator of class c has lower-triangular powers, so
  // the FP32 chain stages of the class leave out the zero blocks
  int class_lower[4] = {0, 0, 0, 0};
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

namespace ssmc {
namespace host {

ssm_status validate_seqs(const ssm_seq_desc* seqs, int32_t n_seq);
// Automatic N: the largest N a sequence can take (its window covers it).
int auto_cap(int64_t L);
// The descriptors with every automatic N at its cap; *any says whether one was.
std::vector<ssm_seq_desc> with_caps(const ssm_seq_desc* seqs, int32_t n_seq, bool* any);
// Builds sequences, operators, work units, info and the workspace layout.
ssm_status build_plan(ssm_plan_s& P, const ssm_seq_desc* seqs, int32_t n_seq, ssm_disc disc,
                      ssm_dtype compute, int32_t with_backward, int32_t ckpt_every,
                      const ssm_tuning* tuning, bool norms_region = false);
// Backward planning: checkpoints, reduction chunks, FP64 gradient workspace.
void plan_backward(ssm_plan_s& P);
// The backward's FP64 GEMM jobs (squaring and discretization adjoints).
void plan_backward_jobs(ssm_plan_s& P);
// Partitioned low-rank stages: eligibility, units, records, compression jobs.
void plan_plr(ssm_plan_s& P);
// After prepare has read the ranks back: the stages that run in PLR form.
void plr_select(ssm_plan_s& P);

}  // namespace host
}  // namespace ssmc
