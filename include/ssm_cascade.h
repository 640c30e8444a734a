/*
 * ssm_cascade.h -- C ABI of the MI355X (gfx950) fast-cascade library.
 *
 * The library applies the transfer function of a discrete linear
 * time-invariant state-space model,
 *     H(z) = C (I - z^{-1} Abar)^{-1} Bbar + D            (eq. (1.3)),
 * in the time domain through the truncated cascade of §2-§3 of Beylkin,
 * "Fast convolution algorithm for state space models" (arXiv 2411.17729):
 * (I - z^{-1} Abar)^{-1} is replaced by the degree-(2^{N+1}-1) polynomial
 * prod_{k=0..N} (I + z^{-2^k} Abar^{2^k})  (eq. (2.2)), so stage k is the
 * shifted update  x_l <- x_l + Abar^{2^k} x_{l-2^k}  for 2^k <= l < L
 * (eqs. (3.2)-(3.4) and the general step of §3), applied to all time steps
 * at once. The input is v_l = Bbar u_l and the output y_l = C x_l + D u_l.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrices are dense and row-major. Sequences are stored time-major:
 *    u of one sequence is an (L x p) block, y an (L x q) block; many
 *    sequences are packed into one buffer at caller-chosen element offsets.
 *  - Pointers documented as "device" point to memory from hipMalloc (or a
 *    caching allocator on top of it) on the device that is current when the
 *    call is made. Pointers documented as "host" are ordinary host memory.
 *  - The caller owns every buffer: parameters, inputs, outputs, gradients and
 *    the workspace. The library never allocates or frees device memory; a
 *    plan is a small host object holding copied descriptors and pointers into
 *    the caller's workspace, which must stay allocated and untouched while the
 *    plan lives.
 *  - Work is enqueued on the given stream (0 = the legacy default stream).
 *    Apart from ssm_cascade_prepare (which synchronizes the stream once to
 *    report numerical failure of the discretization, twice for
 *    SSM_DISC_ZOH), no entry point blocks
 *    the host, so apply, backward and recursion may be captured into a HIP
 *    graph. A plan must be used on one stream at a time.
 *  - Every argument is checked on the host before anything is enqueued;
 *    an invalid argument returns SSM_E_INVALID (or SSM_E_WORKSPACE for a
 *    short workspace) and enqueues nothing. A failed kernel launch returns
 *    SSM_E_HIP. Faults inside kernels surface at the caller's next
 *    synchronization. NaN and Inf propagate; they are not checked.
 *    ssm_last_error() returns a thread-local message describing the most
 *    recent failure. Nothing throws across this ABI.
 *  - Supported sizes: 1 <= m <= 256, 1 <= p <= m, 1 <= q <= m, L >= 1,
 *    0 <= N <= 62 or -30 <= N <= -1 (automatic). Internally the state is
 *    padded to 32, 64, 128 or 256.
 */
#ifndef SSM_CASCADE_H
#define SSM_CASCADE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSM_OK = 0,
  SSM_E_INVALID = 1,      /* bad argument (null pointer, size, offset, dtype) */
  SSM_E_UNSUPPORTED = 2,  /* valid request the library does not implement */
  SSM_E_WORKSPACE = 3,    /* workspace smaller than ssm_cascade_workspace_bytes() */
  SSM_E_HIP = 4,          /* a HIP runtime call or kernel launch failed */
  SSM_E_NOT_PREPARED = 5, /* plan is null or was prepared without what the call needs */
  SSM_E_NUMERIC = 6       /* I - delta/2 A is singular to working precision, or the
                             exponential's scaling is out of range (SSM_DISC_ZOH) */
} ssm_status;

typedef enum {
  SSM_F64 = 0,  /* IEEE binary64 */
  SSM_F32 = 1,  /* IEEE binary32 */
  SSM_BF16 = 2  /* bfloat16 (8-bit significand), round-to-nearest-even */
} ssm_dtype;

typedef enum {
  /* Trapezoidal rule of §1 (the formulas after eq. (1.2)):
   *   Abar = (I - delta/2 A)^{-1} (I + delta/2 A),  Bbar = delta (I - delta/2 A)^{-1} B. */
  SSM_DISC_TRAPEZOID = 0,
  /* A and B are already the discrete Abar and Bbar of eq. (1.2); delta is ignored. */
  SSM_DISC_GIVEN = 1,
  /* Exponential discretization (the choice Abar = exp(delta A) of §5), with
   * Bbar the zero-order hold int_0^delta exp(s A) ds B (the paper's printed
   * "(delta A)^{-1} [exp(delta A) - I] delta A" is read with delta B as its
   * last factor, which it equals for invertible A). Both come from one FP64
   * exponential of [[delta A, delta B], [0, 0]] on the GPU: scaled by 2^-s so
   * that its 1- and infinity-norms are at most 1/2, an 18-term Taylor
   * polynomial, then s squarings. Prepare reads the norms back (a second
   * synchronization of the stream) to fix s per operator; a non-finite norm
   * or s > 60 returns SSM_E_NUMERIC. The backward carries the gradient
   * through it with the adjoint of the exponential's derivative, the
   * upper-right block of the exponential of [[E^T, G], [0, E^T]], formed the
   * same way. */
  SSM_DISC_ZOH = 2
} ssm_disc;

typedef enum {
  SSM_LAUNCH_AUTO = 0,      /* persistent for ragged batches, per stage otherwise */
  SSM_LAUNCH_PER_STAGE = 1, /* one kernel launch per stage */
  SSM_LAUNCH_PERSISTENT = 2 /* one persistent launch for the whole forward pass */
} ssm_launch;

/* Tuning choices of a plan (host memory); a NULL pointer means all defaults.
 * tile_rows[i] is the number of time rows per stage tile for the padded state
 * size 32 << i (i = 0..3): 0 keeps the default, otherwise it must be the
 * default or half of it (the persistent launch always uses the defaults).
 * Defaults: 256, 128, 64, 64 rows for F32/BF16 and 128, 64, 64, 32 for F64. */
typedef enum {
  SSM_STAGE_AUTO = 0,     /* chain where supported, then resident, then tiled */
  SSM_STAGE_TILED = 1,    /* power streamed through LDS in K chunks per row tile */
  SSM_STAGE_RESIDENT = 2, /* power resident in LDS, waves stream 16-row blocks
                             (BF16/FP32 operands and padded m of 64..256 only) */
  SSM_STAGE_CHAIN = 3     /* power resident in LDS; at stages with shift 2^k >= 16
                             each wave walks a column of 16-row blocks spaced 2^k
                             apart and reuses each block's input rows as the next
                             block's shifted operand, so the state is read about
                             once per stage instead of twice (BF16 and FP32 at
                             padded m of 64..256; FP32 m = 256 splits each row's
                             outputs over two workgroups and leaves its last stage
                             to the resident kernel; other stages and sizes use
                             the resident kernel) */
} ssm_stage_kernel;

typedef struct {
  int32_t launch;        /* ssm_launch */
  int32_t tile_rows[4];
  int32_t stage_kernel;  /* ssm_stage_kernel, per-stage launches only */
  /* Leading stages folded into the input pass (per-stage launches and the
   * resident persistent launch): after stages 0..j-1 the state is
   *   x_l = sum_{i < 2^j} Abar^i Bbar u_{l-i} = K_j [u_l; u_{l-1}; ...; u_{l-2^j+1}]
   * with K_j = [Bbar, Abar Bbar, ..., Abar^(2^j - 1) Bbar] built by doubling
   * with the powers, K_{i+1} = [K_i | P_i K_i], i.e. the product of the first j
   * factors of eq. (2.2) applied to Bbar. 0: automatic (the largest j with
   * 2^j p <= m, if at least 2, or 2^j p <= 2 m for the split input pass), -1:
   * none, j > 0: at most j. */
  int32_t input_stages;
  /* Chain kernel: 16-row blocks per wave segment (each segment re-reads one
   * block, its first block's partner). 0: automatic (per-stage launches:
   * blocks of the stage / 2048, at most 8; the persistent launch: blocks of
   * the level / 8192, at most 32), otherwise 1..64. */
  int32_t chain_blocks;
  /* Stage pairs (forward apply with per-stage launches and the chain kernel;
   * BF16 at padded m of 128 and 256): two consecutive stages that are lean for
   * every sequence of a class run as one pass over the state,
   *   w_l = y_l + P_{k+1} y_{l-2^{k+1}},  y_l = x_l + P_k x_{l-2^k},
   * which moves each state row through HBM once for both stages. A workgroup
   * walks a segment of 16-row blocks of one column of stage k; its eight waves
   * split the state entries and exchange each block's x and y (rounded to
   * BF16, the operand type) through LDS. 0: automatic (on where supported),
   * 1: off. */
  int32_t pair_stages;
  /* 16-row blocks per workgroup segment of a stage pair (a segment also reads
   * up to three blocks before it to rebuild its partners). 0: automatic
   * (blocks of the stage / 256, clamped to 8..64), otherwise 4..256. */
  int32_t pair_blocks;
  /* Split input pass (per-stage launches with the chain kernels; BF16 at
   * padded m of 128 and 256, p a multiple of 4): the waves split the state
   * entries and keep the rows of K_j in registers, so the pass folds stages
   * while 2^j p <= 2 m (the resident pass: 2^j p <= m), for classes whose
   * sequences all run stages after the folded ones. 0: automatic (on where
   * supported), 1: off. */
  int32_t input_split;
  /* State kept between the passes of the forward apply (ssm_cascade_apply and
   * its graph; BF16 plans). 0: FP32. 1: BF16 where every pass is the split
   * input pass or a stage pair and the last pair forms y: each pass then reads
   * and writes the state as BF16, still accumulating y_l and w_l in FP32 and
   * rounding them once (to nearest even) when they are written, which halves
   * the state traffic for one more rounding of the state per pass; otherwise
   * FP32 (ssm_plan_info.state_dtype says which). The backward keeps FP32. */
  int32_t state_bf16;
  /* Output pass with the last s stages folded in (forward apply with
   * per-stage launches and the chain kernels; BF16 at padded m of 128 and 256;
   * classes whose sequences all end at the same stage and share the folded
   * input stages, q <= 16, p <= 64). The last s factors of eq. (2.2) multiply
   * out to sum_{j < 2^s} z^{-j 2^k0} Abar^(j 2^k0), k0 the first folded stage,
   * so y_l = sum_j G_j x_{l - j 2^k0} + D u_l with G_j = C Abar^(j 2^k0) (q x m,
   * FP64 during prepare, then rounded once to BF16), x the state after the
   * stages before k0: one pass that reads the state once and writes y in place
   * of the last s stages. At padded m 256 with q <= 8, s = 6: two lags share
   * an MFMA operand (G_{2i} over G_{2i+1}) and the 64 lags are split over
   * the waves of one workgroup, which add their partial outputs in a fixed
   * order (so the result does not depend on timing) before y is stored.
   * 0: automatic (the largest s the LDS holds: 6 at padded m 256 and q <= 8,
   * else 4; 5 at 128; with the stages before it pairing up), -1: off, 2..6:
   * at most that many. */
  int32_t fold_stages;
  /* Persistent launch: an item waits for the items of the level before it
   * (device-scope counters) and gives up after spin_limit sleeps of about 64
   * clocks each (0: the default, 2^25, about a second on MI355X), or at once
   * when another workgroup has given up. A workgroup that gives up skips the
   * rest of its work but still signals it, so the grid always drains and the
   * kernel returns; the give-up is reported by ssm_cascade_device_status. A
   * valid plan never comes near the default; a tiny limit forces the give-up
   * path (for tests). Must be >= 0. */
  int32_t spin_limit;
  /* 1: the workspace leaves out the two state buffers of the forward apply
   * (ssm_cascade_workspace_bytes shrinks by that much), and the plan is
   * applied only through ssm_cascade_apply_noalloc, which takes them from the
   * library's static device scratch; ssm_cascade_apply, _apply_x0,
   * _recursion and _graph_apply then return SSM_E_NOT_PREPARED. Not with
   * with_backward (SSM_E_UNSUPPORTED). 0: the default. */
  int32_t static_state;
  /* 1: the forward apply leaves every sequence's final state x^(N+1) in the
   * state buffers, so that ssm_cascade_apply_state can return the state of
   * its last row (to start the next chunk of a stream from it). The passes
   * that form y without that state (stage pairs, the output fold, BF16 state
   * between passes) are then not used, and the plan launches per stage
   * (SSM_LAUNCH_PERSISTENT returns SSM_E_UNSUPPORTED). 0: the default. */
  int32_t final_state;
  /* Partitioned low-rank powers (§5). d in 1..15: at prepare every power
   * P_k = Abar^{2^k} of a padded size 64..256 is also built in PLR form: the
   * dyadic partition down to 16 x 16 diagonal leaves, each off-diagonal block
   * replaced by Q (Q^T B) with Q from pivoted Gram-Schmidt, of the smallest
   * rank it reaches with ||B - Q Q^T B||_F <= 10^-d (absolute; at most 32 per
   * block). Then ||P_k - PLR(P_k)||_2 <= 2 D 10^-d over the D levels. A stage
   * of the forward apply runs in PLR form where, for every operator of its
   * padded size, the ranks fit and the form takes at most half the matrix-core
   * steps of the dense product; the stage must not be the last of any of those
   * sequences (that stage forms y densely), nor one the input pass covers.
   * ssm_cascade_plr_ranks reports the ranks and the stages chosen. FP32 and
   * FP64 plans, forward only: with_backward, BF16 compute and persistent
   * launches return SSM_E_UNSUPPORTED. 0: off (the default). */
  int32_t plr_digits;
  /* Smallest padded state size: 0 (the default: m padded to 32, 64, 128 or
   * 256) or 64, 128, 256, every operator padded to at least this size. The
   * padding is exact (the padded part of Abar is the identity on a state that
   * no input reaches, and C ignores it). Padding m <= 64 to 128 lets a ragged
   * BF16 batch run every class through the fused passes (input pass, stage
   * pairs, output folds) and keep its state in BF16; the padded rows cost
   * their share of flops and bytes. */
  int32_t min_padded_m;
} ssm_tuning;

/* One sequence of a (possibly ragged) batch. Host memory. */
typedef struct {
  int32_t m, p, q;     /* state, input and output sizes; must equal its parameter set's */
  int32_t N;           /* highest cascade stage: stages k = 0..N, degree 2^{N+1}-1 (eq. (2.2));
                          or automatic, N = -e with e in 1..30: prepare takes the
                          smallest N with |Abar^(2^(N+1))|_F <= 10^-e (the first power
                          the polynomial leaves out, §2, as in the choice of N in §4),
                          at most ceil(log2 L) - 1, where the window covers the
                          sequence and the cascade equals the recursion */
  int64_t L;           /* number of time steps */
  double delta;        /* step size (> 0) of the discretization; ignored for SSM_DISC_GIVEN */
  int32_t param_set;   /* index into the ssm_params array */
  int32_t reserved;    /* must be 0 */
  int64_t u_offset;    /* element offset of this sequence's (L x p) input block */
  int64_t y_offset;    /* element offset of this sequence's (L x q) output block */
} ssm_seq_desc;

/* One parameter set of the continuous model eq. (1.1) (or of the discrete
 * model when SSM_DISC_GIVEN). Device pointers to FP64 row-major matrices:
 * A (m x m), B (m x p), C (q x m), D (q x p). Read only during prepare. */
typedef struct {
  const double* A;
  const double* B;
  const double* C;
  const double* D;
  int32_t m, p, q;
  int32_t reserved; /* must be 0 */
} ssm_params;

/* Gradients of the parameters are written to one flat FP64 device buffer:
 * for each parameter set in order, dA (m x m), dB (m x p), dC (q x m) and
 * dD (q x p), row-major and back to back, i.e. m*m + m*p + q*m + q*p
 * doubles per set (ssm_cascade_param_grad_numel gives the total). */
/* Plan summary, filled by ssm_cascade_plan_info (host memory). */
typedef struct {
  int32_t n_seq, n_ops;      /* sequences; distinct (parameter set, delta) operators */
  int32_t compute;           /* ssm_dtype of the stage contractions */
  int32_t max_stage;         /* largest stage index run by any sequence */
  int64_t total_steps;       /* sum of L over sequences */
  double stage_flops;        /* sum over sequences and stages run as stage contractions
                                (not those folded into the input or output pass) of
                                2 m^2 (L - 2^k) */
  double io_flops;           /* 2 m p L (input) + 2 q (m + p) L (output), summed */
  double stage_bytes;        /* compulsory HBM bytes of the stage launches: per stage and
                                row, read the row once and write it once (the shifted
                                partner is a row of the same stage input); the last stage
                                writes y instead */
  int64_t stage_launches;    /* stage-kernel launches per apply (per-stage mode) */
  int32_t launch;            /* ssm_launch the plan uses (never AUTO) */
  int32_t stage_kernel;      /* ssm_stage_kernel the plan uses (never AUTO) */
  int32_t input_stages;      /* largest number of leading stages folded into the input pass */
  int32_t tile_rows[4];      /* rows per stage tile per padded state size */
  int32_t persistent_grid;   /* workgroups of the persistent launch */
  int64_t persistent_items;  /* work items of the persistent launch */
  int64_t pair_launches;     /* stage-pair launches per apply (counted once in
                                stage_launches; their compulsory bytes, one read
                                and one write of each row for both stages, are
                                part of stage_bytes) */
  double pair_bytes;         /* compulsory HBM bytes of the stage-pair launches */
  double pair_flops;         /* stage flops of the stage-pair launches */
  int32_t state_dtype;       /* ssm_dtype of the state between forward passes */
  int32_t fold_stages;       /* largest number of stages folded into an output pass (0: none) */
  int64_t fold_launches;     /* output-fold launches per apply (counted once in stage_launches;
                                their compulsory bytes, one read of every state row and one
                                write of y, are part of stage_bytes) */
  double fold_bytes;         /* compulsory HBM bytes of the output folds */
  double fold_flops;         /* flops of the output folds: 2 q m per row and lag */
  int32_t plr_stages;        /* (padded size, stage) launches run in PLR form per apply */
  int32_t plr_reserved;
  double plr_flops;          /* flops of those launches over the rows a stage updates:
                                per row 2 (16 mp + sum over the off-diagonal blocks of
                                2 r s) with the ranks found at prepare */
  double plr_dense_flops;    /* the same rows and stages as dense products, 2 mp^2 per row */
  int32_t lower_ops;         /* operators whose Abar (so every power) is lower triangular, as
                                prepare found on the GPU; the FP32 chain stage kernel skips the
                                zero blocks of their powers (stage_flops still counts the dense
                                2 m^2 per row) */
  int32_t lower_reserved;
} ssm_plan_info;

typedef struct ssm_plan_s* ssm_plan;

/* Bytes of device workspace ssm_cascade_prepare needs for this batch.
 * with_backward != 0 reserves what ssm_cascade_backward needs as well: the
 * adjoint ping-pong buffers, per-stage partial sums and the stage-input
 * checkpoints. ckpt_every selects how many stage inputs the backward keeps:
 * 1 keeps every stage input, c >= 2 keeps every c-th one and recomputes the
 * others segment by segment, 0 picks c = ceil(sqrt(number of stages)).
 * Returns 0 if the descriptors are invalid (ssm_last_error() says why). */
size_t ssm_cascade_workspace_bytes(const ssm_seq_desc* seqs, int32_t n_seq,
                                   ssm_disc disc, ssm_dtype compute,
                                   int32_t with_backward, int32_t ckpt_every,
                                   const ssm_tuning* tuning);

/* Discretize, take the powers and pack them (the precomputation of §2-§3:
 * Abar^{2^k} by repeated squaring, k = 0..N). seqs: host array of n_seq
 * descriptors; sets: host array of n_sets ssm_params holding device
 * pointers. compute: SSM_F64, SSM_F32 or SSM_BF16 -- the operand type of the
 * stage contractions (accumulation is FP32 for F32/BF16 and FP64 for F64).
 * Discretization and squaring always run in FP64 on the GPU. Sequences
 * sharing (param_set, delta) share one operator (sharing param_set alone for
 * SSM_DISC_GIVEN). ws: device workspace of ws_bytes >=
 * ssm_cascade_workspace_bytes(seqs, n_seq, disc, compute, with_backward,
 * ckpt_every, tuning) with the same tuning. On success *out receives a new plan (free it with
 * ssm_cascade_destroy). Synchronizes `stream` once at the end (SSM_DISC_ZOH:
 * also once after the norms of delta [A B] are formed). With an automatic N
 * (N < 0 in some descriptor) it runs twice: first with every automatic N at
 * its cap, then, once the norms of the powers are read back (one more
 * synchronization), with the N chosen (ssm_cascade_plan_stages reports
 * them); ssm_cascade_workspace_bytes sizes the workspace for the caps and
 * for every N reached by lowering all automatic N together (in either launch
 * mode), and a choice outside those that needs more returns SSM_E_WORKSPACE
 * with the size in ssm_last_error(). Returns
 * SSM_E_NUMERIC if some I - delta/2 A was singular to working precision, or
 * (SSM_DISC_ZOH) some delta [A B] has a non-finite or too large norm. */
ssm_status ssm_cascade_prepare(const ssm_seq_desc* seqs, int32_t n_seq,
                               const ssm_params* sets, int32_t n_sets,
                               ssm_disc disc, ssm_dtype compute,
                               int32_t with_backward, int32_t ckpt_every,
                               const ssm_tuning* tuning, void* ws, size_t ws_bytes,
                               hipStream_t stream, ssm_plan* out);

/* Forward cascade, eqs. (3.2)-(3.4) and the general step of §3, then
 * y_l = C x_l + D u_l. u: device, u_numel elements of u_dtype (SSM_F64 for
 * an F64 plan; SSM_F32 or SSM_BF16 otherwise). y: device output, y_numel
 * elements of double (F64 plan) or float (F32/BF16 plans). Every sequence's
 * block must lie inside its buffer. */
ssm_status ssm_cascade_apply(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                             size_t u_numel, void* y, size_t y_numel,
                             hipStream_t stream);

/* Reverse-mode derivative of sum(dy * y) for y = apply(u): the adjoint cascade
 * runs the transposed stages in reverse order with reversed shifts,
 *     g_l <- g_l + (Abar^{2^k})^T g_{l+2^k},   k = N..0,
 * recomputing stage inputs from checkpoints, and carries the gradient through
 * the repeated squaring and the discretization. u, dy: device (dy has the
 * layout and element type of y). du: device, u's layout in y's element type
 * (float or double), or NULL. grad_params: device FP64 buffer of
 * grad_numel >= ssm_cascade_param_grad_numel(plan) elements laid out as
 * described above, or NULL; gradients of a set are summed over the
 * sequences that use it, and the buffer is overwritten. Requires a plan
 * prepared with with_backward != 0. */
ssm_status ssm_cascade_backward(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                size_t u_numel, const void* dy, size_t dy_numel,
                                void* du, double* grad_params, size_t grad_numel,
                                hipStream_t stream);

/* ssm_cascade_backward for the apply from an initial state x_{-1} = x0
 * (ssm_cascade_apply_x0 / _apply_state): the initial state enters the
 * forward as the input Abar x0 at row 0 (eq. (1.2) unrolled), so with g =
 * dL/dV^(0) from the adjoint cascade, dL/dx0 = Abar^T g_0, dL/dAbar gains
 * g_0 x0^T, and dL/dC sees the free response through the recomputed
 * states.
 *   x0: device, packed states as for ssm_cascade_apply_x0, or NULL (zero).
 *   dx0: device output in the same layout (the state type), or NULL.
 *   the rest: as ssm_cascade_backward.
 * Errors: as ssm_cascade_backward, and SSM_E_INVALID for a wrong x0_numel
 * or dx0_numel. */
ssm_status ssm_cascade_backward_x0(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                   const void* x0, size_t x0_numel, const void* dy, size_t dy_numel,
                                   void* du, void* dx0, size_t dx0_numel, double* grad_params,
                                   size_t grad_numel, hipStream_t stream);

/* Number of doubles of the flat parameter-gradient buffer of a plan. */
size_t ssm_cascade_param_grad_numel(ssm_plan plan);

/* Forward apply from a nonzero initial state x_{-1} = x0 (eq. (1.2), whose
 * problem statement in §1 takes x_{-1} = 0; ssm_cascade_apply is this with
 * x0 = 0). Unrolled, x_l = Abar^(l+1) x_{-1} + sum_{j<=l} Abar^j Bbar u_{l-j},
 * so x_{-1} enters as one more input Abar x_{-1} at l = 0 and the cascade
 * keeps its lags l < 2^{N+1}: y_l gains C Abar^(l+1) x0 for l < 2^{N+1}, and
 * equals the recursion from x0 whenever L <= 2^{N+1}.
 *   x0: device, the plan's state type (double for SSM_F64 plans, float
 *       otherwise), the sequences' states packed in sequence order, m_s
 *       entries each; x0_numel must be their sum. Read during the call only.
 *   u, y: as for ssm_cascade_apply.
 * Errors: SSM_E_INVALID (x0 NULL or x0_numel wrong, and the checks of
 * ssm_cascade_apply), SSM_E_UNSUPPORTED for persistent plans and plans that
 * keep a BF16 state, SSM_E_HIP on a launch failure. Cost: one extra small
 * launch of min(2^kry, L) dependent FP64 matvecs per sequence (kry: the
 * stages folded into the plan's input pass). */
ssm_status ssm_cascade_apply_x0(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                const void* x0, size_t x0_numel, void* y, size_t y_numel,
                                hipStream_t stream);

/* Forward apply of one chunk of a stream: from the initial state x0 (as
 * ssm_cascade_apply_x0; NULL for x_{-1} = 0), and returning the state of the
 * last row, x_last = x_{L-1} of each sequence (eq. (1.2) unrolled: x_{L-1} =
 * Abar^L x0 + sum_{j<L} Abar^j Bbar u_{L-1-j} when L <= 2^{N+1}). Passing one
 * chunk's x_last as the next chunk's x0 continues the recursion of eq. (1.2)
 * across chunks of at most 2^{N+1} rows each, exactly up to rounding.
 * (Chunks longer than 2^{N+1} rows carry the truncated state of the
 * cascade instead. The truncated operator H_N itself is streamed without
 * any carried state by prepending the previous 2^{N+1} - 1 inputs to each
 * chunk and keeping the last outputs.)
 *   x0: device, the plan's state type (double for F64 plans, float
 *       otherwise), the sequences' states packed in sequence order, m_s
 *       entries each, x0_numel their sum; or NULL (then x0_numel is ignored).
 *   x_last: device output in the same layout, or NULL. Needs a plan
 *       prepared with ssm_tuning.final_state = 1 (SSM_E_NOT_PREPARED
 *       otherwise); may be the same buffer as x0 (x0 is read before x_last
 *       is written, on the same stream).
 *   u, y: as for ssm_cascade_apply.
 * Errors: as ssm_cascade_apply_x0, and SSM_E_INVALID for a wrong x_last_numel. */
ssm_status ssm_cascade_apply_state(ssm_plan plan, const void* u, ssm_dtype u_dtype, size_t u_numel,
                                   const void* x0, size_t x0_numel, void* y, size_t y_numel,
                                   void* x_last, size_t x_last_numel, hipStream_t stream);

/* ssm_cascade_apply without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, checks, kernels and results as
 * ssm_cascade_apply, bit for bit; the two state buffers the passes ping-pong
 * between come from a static device array of the library (64 MiB, reserved
 * on every device the library runs on until the process ends) instead of the
 * plan's workspace, so a plan prepared with ssm_tuning.static_state = 1 needs
 * no workspace for them. The call makes no HIP allocation and records no
 * timing events.
 * Limit: the plan's two state buffers (sum over sequences of L * padded m
 * elements of 4 bytes, 8 for F64 plans, each) must fit in the 64 MiB;
 * otherwise SSM_E_WORKSPACE and nothing is enqueued.
 * Every call on one device shares that device's array and leaves its last
 * contents there: calls that overlap on one device (two streams, two host
 * threads, or a graph replay beside an eager call) race and corrupt each
 * other's results. Serialize them. */
ssm_status ssm_cascade_apply_noalloc(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                     size_t u_numel, void* y, size_t y_numel,
                                     hipStream_t stream);

/* The plain recursion x_n = Abar x_{n-1} + Bbar u_n, y_n = C x_n + D u_n of
 * eq. (1.2) on the GPU (one workgroup per sequence, L dependent steps), for
 * comparison with the cascade. Same arguments as ssm_cascade_apply; runs in
 * FP64 for an F64 plan and FP32 otherwise. It is the full (untruncated)
 * recursion, so it equals the cascade when 2^{N+1} >= L. */
ssm_status ssm_cascade_recursion(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                 size_t u_numel, void* y, size_t y_numel,
                                 hipStream_t stream);

/* Copies the FP64 power Abar^{2^k} of operator `op` (the op-th distinct
 * (param_set, delta) pair in order of first appearance in seqs) into the
 * device buffer dst (m x m row-major, m of that operator), k = 0..N_op.
 * Enqueued on `stream`. For verification of the precomputation. */
ssm_status ssm_cascade_get_power(ssm_plan plan, int32_t op, int32_t k,
                                 double* dst, hipStream_t stream);

/* Copies Bbar (m x p) of operator `op` into dst (device, FP64). */
ssm_status ssm_cascade_get_bbar(ssm_plan plan, int32_t op, double* dst,
                                hipStream_t stream);

/* Synchronizes `stream` and reports whether the last persistent launch of the
 * plan (apply or its graph) gave up a wait for the items it depends on (see
 * ssm_tuning.spin_limit): SSM_E_HIP if it did (its output is not valid; the
 * next apply clears the record), SSM_OK otherwise and for plans that do not
 * launch persistently. Also returns SSM_E_HIP if the synchronization reports
 * an earlier asynchronous failure. */
ssm_status ssm_cascade_device_status(ssm_plan plan, hipStream_t stream);

/* The N of every sequence of the plan (after an automatic choice), into the
 * host array N of n = n_seq entries. */
ssm_status ssm_cascade_plan_stages(ssm_plan plan, int32_t* N, int32_t n);

/* Partitioned low-rank powers (ssm_tuning.plr_digits): for operator `op` and
 * stage k (0..N_op), the ranks of the off-diagonal blocks of P_k found at
 * prepare into the host array ranks of n >= 32 entries, entry
 * 2 (2^(d-1) - 1) + 2 g + side for level d (block size m_pad / 2^d), node g
 * and side 0 (lower block) or 1 (upper block); 33 marks a block whose rank
 * exceeds 32; entries past 2 (2^D - 1) are 0. *used = 1 if the forward apply
 * runs stage k of this operator's padded size in PLR form. SSM_E_UNSUPPORTED
 * for a plan prepared without PLR powers or an operator of padded size 32. */
ssm_status ssm_cascade_plr_ranks(ssm_plan plan, int32_t op, int32_t k, int32_t* ranks, int32_t n,
                                 int32_t* used);

/* Host-side summary of a plan. */
ssm_status ssm_cascade_plan_info(ssm_plan plan, ssm_plan_info* info);

/* Per-launch timing with HIP events recorded on the launch stream.
 * enable != 0 makes later apply/backward/recursion calls record an event pair
 * around every kernel launch (this adds host work; leave it off otherwise).
 * ssm_cascade_timing_read returns, for kernel class `kind`
 * (0 = forward stage, 1 = adjoint stage, 2 = outer-product reduction,
 *  3 = recursion, 4 = forward stage pair, 5 = output fold, 6 = forward stage in
 *  PLR form), the number of timed launches and
 * their summed milliseconds,
 * after synchronizing the events, and clears the record. */
ssm_status ssm_cascade_timing_enable(ssm_plan plan, int32_t enable);
ssm_status ssm_cascade_timing_read(ssm_plan plan, int32_t kind, int64_t* launches,
                                   double* total_ms);

/* HIP graphs of one call. The call is captured on `stream` (which must not be
 * the legacy default stream 0) with the given buffers and instantiated;
 * ssm_cascade_graph_launch replays it on any stream. The plan, the workspace
 * and every buffer must outlive the graph; buffer contents may change
 * between replays. Timing records are not captured. Nothing the library
 * enqueues is a memset: counters are cleared by a kernel, so replays start
 * from the same state. */
typedef struct ssm_graph_s* ssm_graph;

ssm_status ssm_cascade_graph_apply(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                   size_t u_numel, void* y, size_t y_numel,
                                   hipStream_t stream, ssm_graph* out);
ssm_status ssm_cascade_graph_backward(ssm_plan plan, const void* u, ssm_dtype u_dtype,
                                      size_t u_numel, const void* dy, size_t dy_numel,
                                      void* du, double* grad_params, size_t grad_numel,
                                      hipStream_t stream, ssm_graph* out);
ssm_status ssm_cascade_graph_launch(ssm_graph graph, hipStream_t stream);
/* NULL is accepted. */
ssm_status ssm_cascade_graph_destroy(ssm_graph graph);

/* Frees the host plan (not the workspace). NULL is accepted. */
ssm_status ssm_cascade_destroy(ssm_plan plan);

/* Static string for a status code. */
const char* ssm_status_string(ssm_status s);
/* Thread-local detail of the most recent failure on this thread ("" if none). */
const char* ssm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSM_CASCADE_H */
