// Internal declarations shared by the host API and the kernels of the
// fast-cascade library. Not part of the public ABI (include/ssm_cascade.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssmc {

// Element types (same numbering as ssm_dtype).
enum : int32_t { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// One sequence, as the kernels see it.
struct SeqDev {
  int64_t L;
  int64_t x_off;  // element offset of row 0 in every state buffer (rows of mp)
  int64_t u_off;  // element offset of the (L x p) block of u / du
  int64_t y_off;  // element offset of the (L x q) block of y / dy
  int32_t op;     // operator index
  int32_t last;   // last stage index this sequence runs (0 if no stage acts)
  int32_t p, q;
  int32_t kry;    // leading stages folded into the input pass by apply (0: none)
  int32_t reserved;
};

// One operator (a distinct discretized Abar with its Bbar, C, D).
// Offsets are element offsets into the plan's buffers.
struct OpDev {
  int64_t pw;    // FP64 powers: Abar^(2^k) at pw + k*mp*mp (mp x mp, zero padded)
  int64_t pc;    // packed powers in the compute type, same layout
  int64_t pct;   // packed transposed powers (adjoint), or -1
  int64_t bin;   // Bbar   (mp x p)  in the state type
  int64_t cout;  // C      (q x mp)  in the state type
  int64_t dmat;  // D      (q x p)   in the state type
  int64_t ct;    // C^T    (mp x q)  in the state type
  int64_t bt;    // Bbar^T (p x mp)  in the state type
  int64_t dt;    // D^T    (p x q)   in the state type
  int64_t bbar;  // FP64 Bbar (mp x p)
  int64_t minv;  // FP64 (I - delta/2 A)^{-1} (mp x mp)
  int64_t sc_aug, sc_n, sc_b;  // prepare scratch: [M | I] (mp x 2mp), I + hA, delta B
  int64_t kw;    // FP64 K_j = [Bbar, Abar Bbar, ...] (mp x kst, columns beyond 2^j p zero), or -1
  int64_t kc;    // K_j in the compute type, same layout, or -1
  int32_t kry;   // j of this operator (0: none)
  int32_t kdim;  // 2^j p
  int32_t kst;   // row stride of K_j: max(mp, 2^j p)
  int32_t ksplit;  // 1: the split input pass (K_j rows in registers) computes x^(j)
  // backward, FP64 gradient workspace offsets
  int64_t g_dp;    // dL/dP_k, k = 0..N (mp x mp each); becomes the squaring adjoint
  int64_t g_dbb;   // dL/dBbar (mp x p)
  int64_t g_s;     // scratch (mp x mp)
  int64_t g_da;    // dL/dA of this operator (mp x mp)
  int64_t g_db;    // dL/dB of this operator (mp x p)
  int32_t mp, m, p, q, N, set;
  double delta;
  // tail pair (stages cpl - 1 and cpl, every sequence of the operator ending at
  // cpl): C P_cpl, 16 x mp (rows from q on zero), FP64 at cpw and in the
  // compute type at cpc; cpl = -1 if the operator has no tail pair
  int64_t cpw, cpc;
  int32_t cpl;
  // output pass with stages fold_k0 .. fold_k0 + fold_s - 1 folded in (every
  // sequence of the operator ending there): G_j = C Abar^(j 2^fold_k0), j <
  // 2^fold_s, as 16 x mp blocks (rows from q on zero), FP64 at fold_gw and
  // packed in operand order in the compute type at fold_gc; fold_s = 0 if none
  int32_t fold_s;
  int64_t fold_gw, fold_gc;
  int32_t fold_k0;
  // 1: the G_j are packed two lags to an operand (rows 0..7 G_{2i}, rows 8..15
  // G_{2i+1}; q <= 8) for the six-stage fold
  int32_t fold_paired;
  // exponential discretization: scratch of three zn x zn FP64 matrices at zx
  // (zn = m + p; the augmented matrix, then the Taylor and squaring
  // ping-pong), and the squarings zsq chosen from its norm; zx = -1 if none
  int64_t zx;
  int32_t zn, zsq;
  // 1 when Abar, and so every power, is lower triangular (set on the device at
  // prepare from the FP64 Abar): the stage contractions then skip the blocks
  // above the diagonal (below it for the transposed powers of the adjoint)
  int32_t lower;
};

// A row tile of one sequence for the stage kernel.
struct Tile {
  int32_t seq;
  int32_t row0;
};

// Stage kernel flags.
enum : int32_t {
  SF_EPILOGUE = 2,     // at the last stage of the direction, write dst rows
  SF_STORE_AT_EPI = 4, // also store the state rows at the epilogue stage
  SF_NOUPDATE = 8,     // no stage update: pure projection pass over all rows,
                       // prologue/epilogue apply unconditionally
};

struct StageParams {
  const Tile* tiles;
  const SeqDev* seqs;
  const OpDev* ops;
  const void* P;      // packed powers base (compute type)
  const void* small;  // small-matrix base (state type)
  const void* xin;    // state rows read
  void* xout;         // state rows written
  const void* xin_first;  // if set: rows read at a sequence's first stage of the direction
  void* xfinal;           // if set: state rows also stored here at a sequence's last stage
  const void* src;    // u (forward) or dy (adjoint)
  void* dst;          // y (forward) or du (adjoint)
  int32_t src_dtype;  // DT_* of src
  int32_t k;          // stage index
  int32_t adjoint;    // 0: x_l += P_k x_{l-2^k};  1: g_l += P_k^T g_{l+2^k}
  int32_t flags;
  int32_t n_tiles;
  int32_t skip_kry;  // stages below a sequence's kry were done by the input pass
  int32_t kry_override;  // resident input pass: j > 0 writes x^(j) (j <= the sequence's kry) to xout
};

// A range of rows of one sequence for the resident-power stage kernel.
struct ResRange {
  int32_t seq, row0, nrows, reserved;
};

// Work of one chain-kernel workgroup at stage k: segments seg0 .. seg0 + 7 of
// sequence seq (one per wave), each T consecutive 16-row blocks in the
// column-by-column numbering of the stage.
struct ChainUnit {
  int32_t seq, seg0, T, reserved;
};

// Work of one stage-pair workgroup at stages k, k+1: blocks f0 .. f0 + T - 1
// of sequence seq in the column-by-column numbering of stage k.
struct PairUnit {
  int32_t seq, f0, T, reserved;
};

// Work of one output-fold workgroup: columns col0 .. col0 + ncol - 1 (ncol <=
// 4, one per wave) of sequence seq in the numbering of its fold stage.
struct FoldUnit {
  int32_t seq, col0, ncol, reserved;
};

// ---- persistent ragged launch ----
// One row tile of one stage (k >= 0), or of the input projection (k == -1),
// of one sequence. Items are ordered by stage level.
struct PItem {
  int32_t seq, k, row0, mp;
};

struct PersistParams {
  StageParams base;        // seqs, ops, P, small, src, dst, src_dtype, flags
  const PItem* items;
  int32_t n_items;
  int32_t spin_limit;      // sleeps a wait may take before it gives up (see persist_wait)
  int32_t* counters;       // [0]: ticket counter; then (last+2) completion counters per sequence
  const int32_t* cnt_off;  // per sequence: index of its first completion counter
  const int32_t* ntiles;   // per sequence: number of row tiles
  void* x0;
  void* x1;
  int32_t* flag;           // give-up flag (the entry after the last counter)
};

// ---- persistent launch on the resident-power kernels ----
// One work item: the input pass over rows [a, a + b) (kind RI_INPUT, which
// completes level kry - 1 of its sequence), a resident-power stage over rows
// [a, a + b) (RI_RES), or a chain unit with first segment a and b blocks per
// segment (RI_CHAIN). An item of level v waits for every item of level v - 1
// of the same sequence. Items are ordered by level.
enum { RI_INPUT = 0, RI_RES = 1, RI_CHAIN = 2 };
struct RItem {
  int32_t seq, k, kind, a, b, level, tail, reserved;
};
struct RPersistParams {
  StageParams base;            // seqs, ops, P, small, src, dst, src_dtype, flags
  const RItem* items;
  int32_t n_items;
  int32_t spin_limit;          // sleeps a wait may take before it gives up (see persist_wait)
  int32_t* counters;           // [0]: ticket counter; then per sequence and level
  const int32_t* cnt_off;      // per sequence: counter of its level kry - 1
  const int32_t* cnt_target;   // per counter: items of that (sequence, level)
  void* x0;
  void* x1;
  int32_t* flag;               // give-up flag (the entry after the last counter)
};

// Default bound of a persistent item's wait for its predecessors: about one
// second of s_sleep(1) at the MI355X clock, far above any wait a valid plan
// produces (a whole ragged forward pass takes milliseconds).
constexpr int32_t kPersistSpinLimit = 1 << 25;

// One thread of a workgroup waits until *cnt >= target. It gives up after
// `limit` sleeps, or at once when another workgroup has given up (*flag set),
// and then sets *flag. Returns true if the wait ended normally. A workgroup
// whose wait gave up skips its item's work but still signals the item done, so
// every later wait ends too and the grid drains.
__device__ __forceinline__ bool persist_wait(const int32_t* cnt, int32_t target, int32_t* flag,
                                             int32_t limit) {
  if (limit <= 0) limit = kPersistSpinLimit;
  int32_t n = 0;
  while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++n > limit || __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// ---- backward ----
// A chunk of rows of one sequence for the outer-product reductions.
struct RedChunk {
  int32_t seq, row0, nrows, slot;
};

// Row sources of the outer-product reductions.
enum : int32_t { RS_STATE = 0, RS_U = 1, RS_DY = 2 };

// partial[slot] = sum over the chunk's rows l of a_l b_{l-s}^T  (dimA x dimB),
// a_l / b_l taken from a state buffer (width mp), u (width p) or dy (width q).
struct RedParams {
  const RedChunk* chunks;
  const SeqDev* seqs;
  const void* a_base;   // state buffer for RS_STATE
  const void* a_first;  // state buffer read instead at k == seq.last (adjoint start), or null
  const void* b_base;   // state buffer for RS_STATE
  const void* u;        // user input (u_dtype)
  const void* dy;       // user output cotangent (state type)
  int32_t u_dtype;
  int32_t a_kind, b_kind;
  int32_t k;           // b rows are shifted by 2^k; -1: no shift
  int32_t check_last;  // sequences with last < k contribute nothing
  int32_t n_chunks;
  void* partial;        // state type, slot stride slot_stride elements
  int64_t slot_stride;
};

// out[e] (FP64) = sum of partial[slot0 + c][e], c < nslots, e < elems.
struct SumJob {
  int64_t slot0;
  int32_t nslots, elems;
  int64_t slot_stride;
  int64_t out;     // element offset into the FP64 gradient workspace
  int64_t kstride; // added k times (per-stage outputs)
  int32_t kmax;    // the job is skipped for k > kmax
  int32_t reserved;
};

// Sum over the operators of a parameter set and crop of the padding into the
// caller's flat gradient buffer.
struct ScatterJob {
  int32_t op_first, n_ops;  // range in the set-ordered operator list
  int32_t m, mp, p, q;
  int64_t dC, dD;  // FP64 workspace offsets of the set's dC (q x mp) and dD (q x p)
  int64_t out;     // offset of the set's block in the caller's buffer
};

// FP64 GEMM job: C = alpha * op(A) * op(B) + beta * C, row-major.
struct GemmJob {
  const double* A;
  const double* B;
  double* C;
  int32_t M, N, K;
  int32_t lda, ldb, ldc;
  int32_t transA, transB;
  double alpha, beta;
  const int32_t* gate;  // if set, the job runs only where *gate != 0
  // if set and *tri != 0, op(A) and op(B) are triangular as tri_mode says
  // (1: op(A) lower, 2: op(A) upper, 4: op(B) lower, 8: op(B) upper) and the
  // contraction leaves out the K ranges where one of them is zero
  const int32_t* tri;
  int32_t tri_mode;
};

// Rows per workgroup tile of the stage kernel for a padded state size and
// compute type (4 waves, 16x16 MFMA blocks).
__host__ __device__ constexpr int stage_bm(int mp, int ct) {
  return ct == DT_F64 ? (mp == 256 ? 32 : mp == 128 ? 64 : mp == 64 ? 64 : 128)
                      : (mp == 256 ? 64 : mp == 128 ? 64 : mp == 64 ? 128 : 256);
}

// Device pointers of one operator's source parameters (FP64, row-major,
// unpadded: A m x m, B m x p, C q x m, D q x p).
struct OpSrc {
  const double* A;
  const double* B;
  const double* C;
  const double* D;
};

// ---- launchers (defined in the .hip files) ----
// bm: rows per tile of the launch's tile table (stage_bm or half of it).
hipError_t launch_stage(int mp, int ct, int bm, const StageParams& prm, hipStream_t s);
// Input projection into the state buffer xout: Bbar u (forward) or C^T dy
// (adjoint) for every tile of the launch (rows: rows per tile).
hipError_t launch_project(int mp, int state_f64, int rows, const StageParams& prm,
                          hipStream_t s);

hipError_t launch_gemm_f64(const GemmJob* jobs_dev, int n_jobs, int max_m, int max_n,
                           hipStream_t s);
// C = alpha A + beta C per job (B, K, ldb, trans* unused).
hipError_t launch_axpy(const GemmJob* jobs_dev, int n_jobs, int max_m, int max_n,
                       hipStream_t s);

// Builds, per operator, the trapezoid system [I - h A | I] (aug, mp x 2mp),
// I + h A (nmat, mp x mp) and delta*B (bsc, mp x p); for given parameters
// writes Abar into the k = 0 power slot and Bbar into bbar directly.
hipError_t launch_zoh_setup(const OpDev* ops, int n_ops, const OpSrc* src, double* zs, double* zid, int nid,
                            double* norms, double* pw, double* bbar, int max_n, hipStream_t s);
hipError_t launch_disc_setup(const OpDev* ops, int n_ops, const OpSrc* src, int given,
                             double* aug, double* nmat, double* bsc, double* pw,
                             double* bbar, int max_mp, hipStream_t s);

// Gauss-Jordan elimination with partial pivoting of aug -> minv, one
// workgroup per operator, skipped for operators whose tri flag is set (their
// inverse comes from the triangular path). Sets *status to 1 if a pivot is
// negligible.
hipError_t launch_gauss_jordan(const OpDev* ops, int n_ops, double* aug, double* minv,
                               int* status, const int32_t* tri, hipStream_t s);

// Lower-triangular I - h A (the HiPPO matrices of §4 are lower triangular):
// tri[op] = 1 if A has no entry above the diagonal, scale[op] = max |I - h A|.
hipError_t launch_mark_lower(OpDev* ops, int n_ops, const double* pw, hipStream_t s);
hipError_t launch_tri_check(const OpDev* ops, int n_ops, const OpSrc* src, int32_t* tri, double* scale,
                            hipStream_t s);
// Inverses of the 32 x 32 diagonal blocks of the lower-triangular M (left
// half of aug) into minv by forward substitution, zeros right of each block
// row's diagonal block; status |= 1 for a diagonal entry below mp eps scale.
// Only for operators with tri[op] set.
hipError_t launch_tri_diag_inv(const OpDev* ops, int n_ops, int max_mp, const double* aug, double* minv,
                               const int32_t* tri, const double* scale, int* status, hipStream_t s);

// Casts K_j (FP64, mp x mp per operator with kw >= 0) to the compute type.
hipError_t launch_pack_krylov(const OpDev* ops, int n_ops, const double* kw, void* kc, int ct,
                              int max_mp, hipStream_t s);

// Casts the FP64 powers to the compute type (and transposes when want_t),
// and fills the small state-type matrices (Bbar, C, D and transposes).
hipError_t launch_pack(const OpDev* ops, int n_ops, const OpSrc* src, const double* pw,
                       const double* bbar, void* pc, int ct, int want_t, void* small,
                       int state_is_f64, int max_mp, int max_N, hipStream_t s);

// Resident-power stage kernel (BF16/FP32 operands, padded m of 64..256).
bool res_supported(int mp, int ct);
// True when a workgroup holds only part of the state rows (then the stage
// cannot apply the output projection).
bool res_splits_rows(int mp, int ct);
hipError_t launch_stage_res(int mp, int ct, const StageParams& prm, const ResRange* ranges,
                            int n_ranges, hipStream_t s);
// Input pass with the leading kry stages folded in: x^(kry)_l = K u-window_l,
// written to xin (kry even) or xout (kry odd); y at once when kry = last + 1.
hipError_t launch_krylov_res(int mp, int ct, const StageParams& prm, const ResRange* ranges,
                             int n_ranges, hipStream_t s);
// Input pass with the state entries split over the waves and K_j rows in
// registers (BF16, padded m 128 and 256, p = 4 or a multiple of 8, 2^j p of
// 128, 256 or 512 and at most 2 mp, every sequence with stages after j): x^(j)
// into xin (j even) or xout (j odd). All operators of a launch share p and
// 2^j p. units: row ranges; lds: (rows + 2^j - 1) p 2 bytes for the largest
// unit, at most 64 KiB. xb: the state is stored as BF16 (element offsets
// x_off as for FP32, two bytes each).
bool input_split_supported(int mp, int ct, int p, int kdim);
hipError_t launch_input_split(int mp, int ct, int p, int kdim, bool xb, const StageParams& prm,
                              const ResRange* units, int n_units, size_t lds, hipStream_t s);
// Chain-walking stage kernel (stages with 2^k >= 16): BF16 and FP32 at padded
// m of 64..256; FP32 m = 256 splits the output rows over two workgroups and
// has no tail variant (tail launches take the resident or tiled kernel).
bool chain_supported(int mp, int ct);
// tail: some sequence of the launch has its last stage here (the forward
// epilogue or the final-state copy may be due); false selects the lean variant.
// The output y = C x + D u (adjoint: du = Bbar^T g + D^T dy) of the sequences
// whose last stage of the direction is prm.k, from the state rows that stage
// stored in prm.xout; for stage launches that ran without their epilogue
// (FP32 at padded m 256, where a stage's rows are split between workgroups).
// ew: outputs, er: inputs per row (both at most 16).
bool output_proj_supported(int mp, int ct, int ew, int er);
hipError_t launch_output_proj(int mp, const StageParams& prm, const ResRange* ranges, int n_ranges,
                              hipStream_t s);
// tri (FP32 operands; ignored for BF16): 1 when every operator of the launch
// has lower-triangular powers, 2 for the adjoint of such a launch, 0 otherwise
// (a launch with tri != 0 over a power that is not triangular is wrong).
hipError_t launch_stage_chain(int mp, int ct, const StageParams& prm, const ChainUnit* units,
                              int n_units, bool tail, int tri, hipStream_t s);
// Stages prm.k and prm.k + 1 of the forward cascade in one pass (2^k >= 16):
// BF16 at padded m of 128 and 256. Lean: both stages are lean for every
// sequence of the units, prm.xin and prm.xout differ. tail: k + 1 is the last
// stage of every sequence of the units, which get y = C x + D u (q <= 16, p <=
// 256; no state is stored). xb: the state read (and written) is BF16. lds:
// pair_lds(mp, tail, largest T, largest p, largest q).
bool pair_supported(int mp, int ct);
size_t pair_lds(int mp, bool tail, int seg_blocks, int p, int q);
hipError_t launch_stage_pair(int mp, int ct, const StageParams& prm, const PairUnit* units,
                             int n_units, bool tail, bool xb, size_t lds, hipStream_t s);

// Output pass with the stages from o.fold_k0 on folded in (BF16 at padded m
// of 128 and 256, q <= 16, p <= 64; s = 2 .. fold_max_stages(mp)): y = sum_j
// G_j x_{l - j 2^k0} + D u from the state prm.xin. xb: that state is BF16.
// lds: fold_lds(mp, s, largest p, largest q).
int fold_max_stages(int mp);
bool fold_supported(int mp, int ct, int s);
size_t fold_lds(int mp, int s, int p, int q);
hipError_t launch_output_fold(int mp, int ct, int s, bool xb, const StageParams& prm, const FoldUnit* units,
                              int n_units, size_t lds, hipStream_t st);
// Packs the FP64 G_j of every operator with a fold (16 x mp blocks) into the
// compute type in operand order.
hipError_t launch_pack_fold(const OpDev* ops, int n_ops, const double* gw, void* gc, int ct, hipStream_t s);
// Output pass with six stages folded in (padded m 256, q <= 8, p <= 64, BF16):
// one column per workgroup, G_j paired two to an operand and the 64 lags split
// over its eight waves, which sum their partial outputs in LDS before y is
// stored once.
bool fold_wide_supported(int mp, int ct, int q, int p);
size_t fold_wide_lds();
hipError_t launch_output_fold_wide(int mp, int ct, bool xb, int max_p, bool q4, const StageParams& prm,
                                   const FoldUnit* units, int n_units, hipStream_t st);

// Zeroes n int32 counters (a kernel, so that graph capture records no memset).
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);
// One persistent launch that runs every item of the plan's forward pass.
hipError_t launch_persistent(int ct, const PersistParams& pp, int grid, hipStream_t s);
// Persistent launch whose items run the chain, resident and input-pass code
// (BF16 at padded m 64..256, FP32 at 64 and 128: no split rows); lds: dynamic LDS bytes for
// the largest class present (persist_res_lds).
size_t persist_res_lds(int ct, int max_mp);
// Segments per wave of a chain item in that launch (a unit spans 8 times as
// many); an item that ends its sequence (tail) walks one.
int chain_segments_persist(int mp, int ct, bool tail);
hipError_t launch_persist_res(int ct, const RPersistParams& pp, int grid, size_t lds, hipStream_t s);
// Workgroups of the persistent kernel that fit on one compute unit.
int persistent_blocks_per_cu(int ct);

// dL/dP_k between two FP32 state buffers (a_kind = b_kind = RS_STATE), padded m 64..256.
hipError_t launch_outer_ss(int mp, const RedParams& prm, hipStream_t s);
// dL/dP_k on the BF16 matrix cores (plans computing in BF16), mp of 128 and 256
hipError_t launch_outer_bf16(int mp, const RedParams& prm, hipStream_t s);
// outer products with one side at most 16 wide (dy or u against a state, dy
// against u): rows read once, coalesced, sums per thread
hipError_t launch_outer_thin(int mp, int state_f64, const RedParams& prm, hipStream_t s);
hipError_t launch_outer(int mp, int state_f64, const RedParams& prm, int tiles_y,
                        hipStream_t s);
hipError_t launch_sum(const SumJob* jobs, int n_jobs, int max_elems, int k,
                      const void* partial, int state_f64, double* out, hipStream_t s);
hipError_t launch_scatter(const ScatterJob* jobs, int n_jobs, const int32_t* set_ops,
                          const OpDev* ops, const double* gws, double* out, int max_mp,
                          hipStream_t s);

// Initial state: adds Abar^(l+1) x0 to rows l < min(2^kry, L) of each sequence
// of padded size mp_class in buffer kry % 2 (after the first pass of an apply),
// or C Abar^(l+1) x0 to those rows of y where that pass formed y (kry = last + 1);
// x0, the buffers, the small matrices and y in the plan's state type (FP64
// when f64, else FP32).
hipError_t launch_inject_x0(int mp_class, bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops,
                            const double* pw, const void* x0, void* buf0, void* buf1, const void* small,
                            void* y, bool keep_state, hipStream_t st);
// Frobenius norms of every operator's powers P_0..P_N (automatic N).
hipError_t launch_power_norms(const OpDev* ops, int n_ops, int max_N, const double* pw, double* norms,
                              hipStream_t s);
// Adds Abar x_{-1} to row 0 of V^(0) (the backward's recomputed input).
hipError_t launch_input_x0(int mp_class, bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops,
                           const double* pw, const void* x0, void* v0, hipStream_t st);
// dL/dx_{-1} = Abar^T g_0 into dx0 (nullable) and g_0 x_{-1}^T added to
// dL/dP_0 in the FP64 gradient workspace G (nullable), g0 the buffer holding
// dL/dV^(0).
hipError_t launch_x0_grads(bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops, int n_ops, const double* pw,
                           const void* x0, const void* g0, void* dx0, double* G, hipStream_t st);
// Row L - 1 of each sequence's final state, left by a plan with the final
// state kept in buffer (last + 1) mod 2, packed into x_last (m entries per
// sequence, in sequence order), in the plan's state type.
hipError_t launch_gather_last(bool f64, const SeqDev* seqs, int n_seq, const OpDev* ops, const void* buf0,
                              const void* buf1, void* x_last, hipStream_t st);
hipError_t launch_recursion(int mp, int ct, const SeqDev* seqs, int n_seq, const OpDev* ops,
                            const double* pw, const double* bbar, const void* u,
                            int u_dtype, void* xout, hipStream_t s);

// Raises the dynamic LDS limit of `kernel` to at least `bytes` on the current
// device. The limit is a per-device function attribute, so the setting is
// remembered per (kernel, device); safe to call from several threads.
hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes);

// The library's static device scratch (state buffers of the allocation-free
// apply): its size, and its address on the current device (looked up once
// per device).
size_t static_scratch_bytes();
hipError_t static_scratch(void** out);

}  // namespace ssmc
