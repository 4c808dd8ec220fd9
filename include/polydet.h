/*
 * polydet: exact determinants of matrices of multivariate integer polynomials on MI355X.
 *
 * The operation is the one of Wei & Chen, "Optimized Multivariate Polynomial Determinant
 * on GPU" (arXiv 2010.12117), Algorithm 1: for an n x n matrix M whose entries are
 * polynomials in x1..xk with integer coefficients, return det M in Z[x1..xk] exactly.
 * The method is modular (Section 2): for each word-size prime p with a large power-of-two
 * root of unity (equation "primes"), every entry is evaluated on a grid of roots of unity
 * (FFT), a determinant is taken at every grid point over Z/pZ (DET, the role of
 * Algorithm 3), the determinant polynomial mod p is interpolated (IFFT, Section 3.3), and
 * the integer coefficients are rebuilt by mixed-radix conversion (CRT, Section 3.4 and
 * Algorithm 4).
 *
 * Conventions of this interface
 * -----------------------------
 * Input coefficients: int64, C order [n][n][deg[0]+1]...[deg[k-1]+1]. Entry (i, j) is the
 *   dense coefficient box of a polynomial, first variable slowest, exactly the encoding of
 *   Section 2's worked example (F = 1 + 2x + 3xy + 4x^2 + 5y^2 -> [1,0,5,2,3,0,4,0,0]).
 *   Any int64 is accepted, INT64_MIN included. nvars = 0 means an integer matrix.
 * Degree bound: D[v] = n * deg[v], an upper bound on the determinant's degree in x_v.
 * Grid: N[v] = next power of two >= D[v] + 1 (the paper rounds degrees up to powers of two,
 *   Section 2; interpolation needs D[v] + 1 distinct nodes, Theorem 1), G = prod N[v].
 * Primes: p in (2^29, 2^30) with p = 1 mod 2^16, in descending order ("9-digit" primes
 *   of the form c * 2^q + 1, Section 2; below 2^30 the elimination may leave its entries
 *   unreduced in [0, 2p) between steps). The count pn is the least with
 *   (p_0 ... p_{pn-1})^2 > 4 B^2, where B^2 = min(prod_i sum_j |a_ij|_1^2,
 *   prod_j sum_i |a_ij|_1^2) bounds the squared coefficients of det M (Hadamard's
 *   inequality on 1-norms; the paper says only that the bound is easily computed).
 * Output: uint32 limbs [D[0]+1]...[D[k-1]+1][limbs], coefficient of x^e at the multi-index
 *   e (first variable slowest), each coefficient a little-endian two's-complement integer
 *   of `limbs` 32-bit words, recovered in the symmetric range (-(M-1)/2, (M-1)/2] with
 *   M = p_0 ... p_{pn-1}. Coefficients above the true degree are zero.
 *
 * Ownership: the caller owns coefficient, output and workspace buffers (device memory
 *   unless stated). A plan owns its device constant tables (allocated by polydet_plan*,
 *   freed by polydet_plan_destroy). Plans are immutable after creation; solves on one plan
 *   may run concurrently on different streams when each has its own workspace and output.
 * Errors: argument and shape errors return synchronously and enqueue nothing. Solves are
 *   asynchronous on `stream`; a launch failure returns POLYDET_EDEVICE, a later device
 *   fault shows at the caller's stream synchronisation. polydet_last_error() returns a
 *   message for the calling thread's last failure.
 */
#ifndef POLYDET_H
#define POLYDET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum polydet_status {
  POLYDET_OK = 0,
  POLYDET_EINVAL = 1,        /* bad argument, shape or buffer size */
  POLYDET_EUNSUPPORTED = 2,  /* beyond the library's limits (see polydet_limits) */
  POLYDET_ENOMEM = 3,        /* host or device allocation failed */
  POLYDET_EDEVICE = 4,       /* HIP error; message in polydet_last_error() */
  POLYDET_ECANCELLED = 5
} polydet_status;

#define POLYDET_MAX_VARS 8

/* Shape of one matrix. coeff_bits: every |coefficient| <= 2^coeff_bits (0..63); used for
 * the worst-case bound when a plan is made without the coefficients. */
typedef struct polydet_shape {
  int32_t n;
  int32_t nvars;
  int32_t deg[POLYDET_MAX_VARS];
  int32_t coeff_bits;
} polydet_shape;

/* POLYDET_UNFUSED_EVAL: write the full evaluation tensor (off_eval) and run the
 * elimination from it, in the paper's stage order. By default the evaluation along the
 * first variable is fused into the elimination kernel and that tensor is never written
 * (off_eval is then SIZE_MAX). Results are identical either way. */
#define POLYDET_UNFUSED_EVAL ((uint32_t)1u)
/* POLYDET_BATCH_PLAIN (batch plans): solve the matrices one after another with the
 * single-matrix launches, instead of the default batched launches (matrices grouped into
 * chunks that fit the workspace; per chunk one persistent launch per stage and one per
 * matrix order for the elimination). Results are identical either way. */
#define POLYDET_BATCH_PLAIN ((uint32_t)2u)
/* POLYDET_DET_LEFT_LOOKING / POLYDET_DET_EXCHANGE: choose the elimination form. By default
 * (and with EXCHANGE) the exchanging kernel computes every determinant. LEFT_LOOKING, for
 * orders up to 16 when the first variable is evaluated inside the elimination, first runs a
 * left-looking pass (one lane per matrix, only the pivot rows in registers, no row
 * exchanges); the points where it meets a zero pivot are then recomputed by the exchanging
 * kernel. Results are identical either way. */
#define POLYDET_DET_LEFT_LOOKING ((uint32_t)4u)
#define POLYDET_DET_EXCHANGE ((uint32_t)8u)
/* The workspace budget of one chunk of a batched solve is 16 GiB, or the value of the
 * environment variable POLYDET_BATCH_BUDGET_MB (in MiB) read when the plan is made; a single
 * matrix larger than the budget forms a chunk of its own. Consecutive chunks run side by
 * side: each chunk takes half the budget and alternates between the two halves of the
 * workspace, even chunks on the caller's stream and odd ones on a stream of the plan's own
 * (default priority; forked from and joined back into the caller's stream by events, so a
 * captured solve stays one graph), so that one chunk's memory-bound passes overlap the next
 * chunk's elimination. With the environment variable POLYDET_BATCH_STREAMS = 1 (read when the
 * plan is made) every launch runs on the caller's stream, in chunks of the whole budget.
 * Plans made with POLYDET_STAGE_TIMING run every launch on the caller's stream.
 * Interpolation passes of 32 to 256 points along a contiguous axis take their transform in
 * registers (one LDS exchange per pass); the environment variable POLYDET_INTT_REGISTERS = 0,
 * read once per process, keeps every pass in the LDS-staged form. Results are identical. */
/* Plan flags. POLYDET_FORCE_PN(x): use exactly x primes (x >= the number the bound needs,
 * else EINVAL). POLYDET_PRIME_OFFSET(x): skip the first x primes of the table (a disjoint
 * prime set; the result does not depend on it). */
#define POLYDET_FORCE_PN(x) ((uint32_t)((x) & 0xFFF) << 8)
/* POLYDET_DET_LANES_LOG2(x): 2^x lanes cooperate on one determinant (x in 0..4) instead
 * of the default for the order; EUNSUPPORTED if no kernel is compiled for that pair. */
#define POLYDET_DET_LANES_LOG2(x) ((uint32_t)(((x) + 1) & 0xF) << 4)
#define POLYDET_PRIME_OFFSET(x) ((uint32_t)((x) & 0x3FF) << 20)
/* POLYDET_HOST_ONLY: compute the plan on the host and upload nothing (no GPU needed); the
 * plan can be queried but not solved (polydet_solve* return EINVAL). */
#define POLYDET_HOST_ONLY ((uint32_t)1u << 31)
/* POLYDET_STAGE_TIMING: every solve of the plan records HIP events on its stream around
 * each stage (read by polydet_stage_times). Solves of such a plan must not overlap. */
#define POLYDET_STAGE_TIMING ((uint32_t)1u << 30)

/* reduce, evaluate, determinants (the elimination kernels: numerator and denominator per
 * point), finalize (det = num / den), interpolate, reconstruct. When the matrix has
 * variables the division is done by the first interpolation pass as it loads the points, and
 * the finalize stage is empty (its time is counted in interpolate). */
#define POLYDET_NUM_STAGES 6

/* What a plan needs and produces. Workspace offsets (bytes) locate the intermediate stages
 * for inspection after a solve on the same stream has completed:
 *   off_eval : uint32 [pn][n*n][G]  entry values at the grid points, Montgomery form
 *              (written only by plans made with POLYDET_UNFUSED_EVAL or with nvars = 0)
 *              (x * 2^32 mod p); point index = natural multi-index (j_1 slowest), node
 *              (w_1^j_1, ..., w_k^j_k) with w_v = g^((p-1)/N[v]), g the least primitive
 *              root mod p;
 *   off_detv : uint32 [pn][G]        numerator of the determinant at each grid point and
 *   off_den  : uint32 [pn][G]        its denominator (never 0), both Montgomery form: the
 *              determinant mod p at the point is num / den (the elimination takes one
 *              inverse per point, in the next stage);
 *   off_coef : uint32 [pn][ncoeff]   coefficients of det M mod p, Montgomery form, times G
 *              (the interpolation's 1/G is applied by the reconstruction); for nvars = 0,
 *              ncoeff = 1 and this is the determinant residue itself.
 * Every stage reads only the outputs of earlier stages, so any stage of a finished solve can
 * be run again on the same workspace (polydet_solve_stages) with the same result. */
typedef struct polydet_plan_info {
  int32_t n, nvars;
  int32_t deg[POLYDET_MAX_VARS];
  int32_t D[POLYDET_MAX_VARS];
  int32_t N[POLYDET_MAX_VARS];
  int64_t G;          /* grid points per prime */
  int64_t ncoeff;     /* prod (D[v] + 1): output coefficients */
  int64_t nterms;     /* prod (deg[v] + 1): input coefficients per entry */
  int32_t pn;         /* primes */
  int32_t limbs;      /* 32-bit limbs per output coefficient */
  int32_t det_lanes;  /* lanes that cooperate on one determinant */
  int32_t det_sign;   /* +1 or -1: see row_order */
  size_t in_bytes;    /* 8 * n * n * nterms */
  size_t out_bytes;   /* 4 * ncoeff * limbs */
  size_t workspace_bytes;
  size_t off_eval, off_detv, off_coef;
  /* The kernels work on the matrix with its rows reordered so that no pivot is zero for
   * structural reasons (from the zero entries of host_coeffs; identity without them): row i
   * of that matrix is input row row_order[i] (i < n). Stage values at off_eval and off_detv
   * refer to the reordered matrix, whose determinant is det_sign times det M. */
  uint8_t row_order[32];
  int32_t det_left_looking; /* 1 if a left-looking pass runs before the exchanging kernel */
  int32_t prime_group;      /* primes per pass of S1-S4 (pn unless the workspace is capped) */
  size_t coef_bytes;        /* 4 * pn * ncoeff: the coefficient residues at off_coef, prime
                             * major ([pn][ncoeff], Montgomery form, factor G left in) */
  size_t off_den;           /* see above */
  int64_t nslots;           /* entries that are reduced and evaluated: with host_coeffs, the
                             * distinct nonzero entries (entries with equal coefficient boxes,
                             * as in Sylvester matrices, are evaluated once); otherwise n*n */
  double predicted_ms;      /* predicted device time of polydet_solve on this plan, from the
                             * rates installed when the plan was built (polydet_set_rates) */
  int32_t grid_slabs;       /* 1, or (capped plans where one prime does not fit) the number of
                             * slabs of the grid along the second variable that S2 and S3 of
                             * one prime run in turn (Section 2: the grid is cut evenly) */
} polydet_plan_info;

typedef struct polydet_plan_s* polydet_plan_t;

/* Build a plan for one matrix shape.
 * host_coeffs: NULL, or the int64 coefficients on the host in the input layout. Without
 *   them the plan holds for every matrix of the shape whose coefficients are at most
 *   2^coeff_bits in absolute value. With them the plan is specialised to those coefficients:
 *   the bound B comes from their 1-norms (fewer primes), their zero entries are skipped by
 *   the kernels (never read), and the rows are reordered around structurally zero pivots
 *   (row_order, det_sign). Such a plan is valid only for matrices with exactly that zero
 *   pattern whose entries' 1-norms are no larger; solving any other coefficient tensor with
 *   it returns a wrong determinant, which polydet_solve cannot detect. For a valid input
 *   the result does not depend on the choice: only pn and limbs do.
 * Returns EINVAL for n < 1, nvars outside 0..8, a negative degree or coeff_bits outside
 * 0..63; EUNSUPPORTED beyond polydet_limits; EDEVICE/ENOMEM when uploading tables fails.
 * The plan's tables live on the device that is current when it is built. */
polydet_status polydet_plan(const polydet_shape* shape, const int64_t* host_coeffs,
                            uint32_t flags, polydet_plan_t* out);

/* polydet_plan with a cap on the workspace of one solve (bytes; 0: no cap). When the solve
 * of all pn primes at once needs more, the plan takes the primes in groups of
 * info.prime_group, the largest that fits: S1-S4 (reduce, evaluation, determinants,
 * interpolation) run group by group on the stream, each group leaving its coefficient
 * residues in the workspace, and the reconstruction runs once at the end (the paper solves
 * one prime at a time; Algorithm 1). When even one prime does not fit, the plan also cuts
 * each prime's grid into info.grid_slabs slabs along the second variable (the least number,
 * a power of two, that fits; Section 2 cuts the grid evenly into chunks): the evaluation over
 * that variable and the determinants run slab by slab, and only one slab's evaluated entries
 * are held at a time. Results are identical to the uncapped plan. EUNSUPPORTED if one prime
 * does not fit even in slabs (or the plan cannot be slabbed: fewer than two variables, or the
 * unfused evaluation); EINVAL with POLYDET_STAGE_TIMING when the cap splits the primes or the
 * grid. */
polydet_status polydet_plan_capped(const polydet_shape* shape, const int64_t* host_coeffs,
                                   uint32_t flags, size_t max_workspace_bytes,
                                   polydet_plan_t* out);

/* Build one plan for `count` matrices of possibly different shapes, solved together by
 * polydet_solve_batch. host_coeffs: NULL or an array of `count` host pointers (each may be
 * NULL). Index i of polydet_plan_query refers to matrix i. */
polydet_status polydet_plan_batch(const polydet_shape* shapes, int32_t count,
                                  const int64_t* const* host_coeffs, uint32_t flags,
                                  polydet_plan_t* out);

/* Plan information; for a batch plan `index` selects the matrix (0 for a single plan). For
 * a batch plan, workspace_bytes is the workspace of the whole batch. */
polydet_status polydet_plan_query(polydet_plan_t plan, int32_t index, polydet_plan_info* out);

/* The primes of matrix `index` (host array of at least pn entries). */
polydet_status polydet_plan_primes(polydet_plan_t plan, int32_t index, uint32_t* out,
                                   int32_t capacity);

/* Solve one matrix (plan made by polydet_plan).
 * d_coeffs: device int64 coefficients (in_bytes); d_out: device uint32 limbs (out_bytes);
 * d_workspace: device scratch of at least workspace_bytes, 256-byte aligned; stream: a
 * hipStream_t (NULL = the default stream). Asynchronous. */
polydet_status polydet_solve(polydet_plan_t plan, const int64_t* d_coeffs, uint32_t* d_out,
                             void* d_workspace, size_t workspace_bytes, void* stream);

/* Size of the library's own workspace for polydet_solve_noalloc (128 MiB per device). */
#define POLYDET_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* polydet_solve without a caller's workspace and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The workspace is a device array of the library,
 * POLYDET_NOALLOC_SCRATCH_BYTES on every device it runs on, held until the process ends;
 * its address is looked up on the first call on each device. The caller still passes the
 * coefficients and the output (as for polydet_solve). Every call on one device shares that
 * array and leaves its contents behind: calls that overlap on one device (several streams or
 * threads) race on it and must be ordered by the caller. EINVAL when the plan's
 * workspace_bytes exceeds POLYDET_NOALLOC_SCRATCH_BYTES (nothing is enqueued); otherwise as
 * polydet_solve. */
polydet_status polydet_solve_noalloc(polydet_plan_t plan, const int64_t* d_coeffs,
                                     uint32_t* d_out, void* stream);

/* Solve every matrix of a batch plan.
 * d_coeffs: device int64 buffer holding every matrix's coefficients; coeff_offsets[i]
 * (host, in int64 elements) is where matrix i starts. d_out: device uint32 buffer;
 * out_offsets[i] (host, in uint32 elements) is where matrix i's limbs start. Outputs of
 * different matrices must not overlap. The offsets are copied to the device on the stream
 * when they differ from the previous call's; with unchanged offsets the solve only enqueues
 * kernels (it can be captured in a HIP graph). Solves of one batch plan must not overlap. */
polydet_status polydet_solve_batch(polydet_plan_t plan, const int64_t* d_coeffs,
                                   const int64_t* coeff_offsets, uint32_t* d_out,
                                   const int64_t* out_offsets, void* d_workspace,
                                   size_t workspace_bytes, void* stream);

/* Stages [stage_begin, stage_end) of polydet_solve, numbered as in polydet_stage_times
 * (0 reduce, 1 evaluate, 2 determinants, 3 finalize, 4 interpolate, 5 reconstruct), for a
 * single-matrix plan that solves all its primes at once (prime_group == pn). The stages before
 * stage_begin must have run on this workspace (with the same coefficients) earlier on the
 * stream; running stages [0, s) and then [s, 6) gives exactly polydet_solve's result, and a
 * stage may be run again (each reads only earlier stages' outputs), e.g. to time one kernel
 * by itself. d_coeffs is read only when stage 0 is included, d_out written only when stage 5
 * is. With POLYDET_STAGE_TIMING the call counts as one solve whose stages outside the range
 * took no time. EINVAL for an empty or out-of-range interval, a batch or capped plan. */
polydet_status polydet_solve_stages(polydet_plan_t plan, int32_t stage_begin, int32_t stage_end,
                                    const int64_t* d_coeffs, uint32_t* d_out, void* d_workspace,
                                    size_t workspace_bytes, void* stream);

/* The solve of a single-matrix plan in two parts, for callers that checkpoint, resume or
 * cancel long solves between primes:
 *   polydet_solve_primes runs S1-S4 for primes [prime_begin, prime_end) (0 <= begin < end
 *   <= pn; any split) and leaves their coefficient residues at workspace offset
 *   info.off_coef + 4 * ncoeff * i for prime i; it does not touch the other primes' slots.
 *   polydet_reconstruct runs S5 (Section 3.4, Algorithm 4) from the slots of all pn primes
 *   and writes the output limbs as polydet_solve does.
 * Calling polydet_solve_primes for every prime, in any order and in any number of calls,
 * then polydet_reconstruct, gives exactly polydet_solve's result. The coefficient region
 * (info.coef_bytes at info.off_coef) is all the state between calls: a caller may copy it
 * out after some primes, and later copy it into another workspace and go on with the rest.
 * Both are asynchronous on `stream`; argument errors are EINVAL (batch plans included). */
polydet_status polydet_solve_primes(polydet_plan_t plan, const int64_t* d_coeffs,
                                    int32_t prime_begin, int32_t prime_end, void* d_workspace,
                                    size_t workspace_bytes, void* stream);
polydet_status polydet_reconstruct(polydet_plan_t plan, void* d_workspace,
                                   size_t workspace_bytes, uint32_t* d_out, void* stream);

/* Device time per stage of the solves of a plan made with POLYDET_STAGE_TIMING (the
 * paper's tables report the same split: FFT, DET, IFFT, CRT). Waits for the recorded
 * solves, writes the summed milliseconds of each stage (POLYDET_NUM_STAGES of them, in the
 * order listed there) to ms[] and the number of solves to *solves, and resets the sums.
 * Single-matrix plans record an event at each stage boundary. Batch plans (batched launches)
 * record an event before and after every launch and add its time to the stage of its kind
 * (matrices solved one by one after the batched launches are not included). EINVAL if the
 * plan was made without the flag. */
polydet_status polydet_stage_times(polydet_plan_t plan, double ms[POLYDET_NUM_STAGES],
                                   int64_t* solves);

void polydet_plan_destroy(polydet_plan_t plan);

const char* polydet_status_string(polydet_status status);

/* Message describing the calling thread's most recent failure ("" if none). */
const char* polydet_last_error(void);

/* Limits of the library: maximum n, nvars, N[v] and pn. Any pointer may be NULL. */
/* Launch-mapping table for the elimination kernel, per class c and matrix order n (1..32;
 * index 0 is unused). Class 0: the first variable has 2 to 4 coefficients (its evaluation is
 * paired across the wave's halves, two terms per lane); class 1: any other matrix with at
 * least one variable (5 or 6 coefficients are paired too, three terms per lane).
 * An entry of 0 keeps the built-in choice; flags given to polydet_plan override the table.
 *   lanes         lanes that share one matrix: 1, 2, 4, 8 or 16 (the pairs the build
 *                 compiles: 1 for n <= 12, 2 for 2..16, 4 for 4..24, 8 for n >= 8, 16 for
 *                 n >= 16)
 *   left_looking  1: left-looking pass and repair (n <= 16); 2: the exchanging kernel alone
 *   tile_points   upper limit on the points per LDS tile of a block (Q): 1, 2, 4, 8 or 16
 * The table is process-wide and read when a plan is built; plans built earlier keep their
 * mapping. It is chosen by measurement (the package's autotuner); no choice in it changes a
 * result. */
#define POLYDET_TUNE_ORDERS 33
typedef struct polydet_tuning {
  int32_t lanes[2][POLYDET_TUNE_ORDERS];
  int32_t left_looking[2][POLYDET_TUNE_ORDERS];
  int32_t tile_points[2][POLYDET_TUNE_ORDERS];
} polydet_tuning;

/* Install a table (copied), or the built-in choices with NULL. EINVAL, and no change, if an
 * entry is outside the values above or names a lanes/order pair the build does not compile. */
polydet_status polydet_set_tuning(const polydet_tuning* table);
/* The table in use (all zeros when none is installed). EINVAL for NULL. */
polydet_status polydet_get_tuning(polydet_tuning* out);

/* Rates of the running-time prediction (Section 5, equation predictRunningTime, which
 * predicts a solve from the prime count, the entries, the mean time to transform one entry
 * and the replication factor of repeated entries; here every stage gets a term):
 *   predicted = launches * launch_us
 *             + (8 nslots T + 4 pn nslots T) / reduce_bytes_per_s
 *             + sum over evaluation passes of 4 pn nslots (input + output box) / eval_bytes_per_s
 *             + pn G (n-1) n (2n-1) / 6 / det_updates_per_s[class][n]
 *             + sum over interpolation passes of 4 pn (input + output [+ denominators])
 *               / intt_bytes_per_s
 *             + ncoeff (pn (pn+1) / 2 + pn limbs) / garner_ops_per_s
 * with T = prod (deg[v] + 1), class as in polydet_tuning. A value of 0 keeps the built-in rate.
 * The table is process-wide and read when a plan is built; it is measured on the GPU by the
 * package's calibration. It changes no result. */
typedef struct polydet_rates {
  double det_updates_per_s[2][POLYDET_TUNE_ORDERS];
  double reduce_bytes_per_s;
  double eval_bytes_per_s;
  double intt_bytes_per_s;
  double garner_ops_per_s;
  double launch_us;
} polydet_rates;

/* Install a rate table (copied; NULL restores the built-in rates). EINVAL for a negative or
 * non-finite entry. */
polydet_status polydet_set_rates(const polydet_rates* rates);
/* The table in use (built-in values where none was installed). EINVAL for NULL. */
polydet_status polydet_get_rates(polydet_rates* out);

void polydet_limits(int32_t* max_n, int32_t* max_vars, int32_t* max_grid_per_var,
                    int32_t* max_primes);

#ifdef __cplusplus
}
#endif

#endif /* POLYDET_H */
