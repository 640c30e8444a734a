// Planning of the fast-cascade library (host only): validation of the batch,
// operators, the work units of every kernel family, the workspace layout,
// the backward's jobs and the partitioned low-rank stages. Shared by
// ssm_cascade_workspace_bytes and ssm_cascade_prepare.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace ssmc {
namespace host {

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
                      const ssm_tuning* tuning, bool norms_region) {
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
  // squaring adjoint: G_k += G_{k+1} P_k^T + P_k^T G_{k+1}, k = N-1..0; where
  // prepare marked the operator's powers lower triangular, P_k^T is upper
  // triangular and the products skip its zero K ranges
  const OpDev* ops_d = reinterpret_cast<const OpDev*>(P.ws + P.r_meta.off + P.m_ops);
  for (int k = P.max_N - 1; k >= 0; --k) {
    for (int half = 0; half < 2; ++half) {
      int start = (int)P.bjobs.size();
      for (size_t oi = 0; oi < P.ops.size(); ++oi) {
        const OpDev& o = P.ops[oi];
        if (o.N <= k) continue;
        const int64_t mm = (int64_t)o.mp * o.mp;
        double* Gk = G + o.g_dp + k * mm;
        double* Gk1 = Gk + mm;
        double* Pk = pw + o.pw + k * mm;
        const int32_t* low = &ops_d[oi].lower;
        if (half == 0)
          P.bjobs.push_back(
              GemmJob{Gk1, Pk, Gk, o.mp, o.mp, o.mp, o.mp, o.mp, o.mp, 0, 1, 1.0, 1.0, nullptr, low, 8});
        else
          P.bjobs.push_back(
              GemmJob{Pk, Gk1, Gk, o.mp, o.mp, o.mp, o.mp, o.mp, o.mp, 1, 0, 1.0, 1.0, nullptr, low, 2});
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

}  // namespace host
}  // namespace ssmc
