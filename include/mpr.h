/*
 * mpr.h -- C ABI of libmpr: exact (min,+) matrix powers on AMD Instinct
 * MI355X (gfx950) for the Roman domination number of cylinders P_m x C_n,
 * after Martinez, Garzon and Puertas, "Powers of large matrices on GPU
 * platforms to compute the Roman domination number of cylindrical graphs"
 * (arXiv 2409.17658).
 *
 * Storage.  Matrices are row-major uint16 with a leading dimension (ld, in
 * elements, ld >= number of columns).  0xFFFF (MPR_INF) is +infinity, the
 * absorbing element of the (min,+) semiring of Section 3.  A matrix that
 * enters a product must have every finite entry <= MPR_FMAX (0x7FFF): the
 * kernels add with unsigned saturation, so every finite sum is <= 0xFFFE and
 * can never be mistaken for infinity.
 *
 * Canonical form of a power.  A power P = A^k is kept as (N, R): R[i] is the
 * least finite entry of row i of P (int64), N = P - R row-wise (so every
 * non-empty row of N has minimum 0).  A row of P with no finite entry has
 * R[i] = MPR_ROW_NONE and an all-infinite row in N.  By the scalar rule of
 * Section 3 ((alpha (x) A) (x) B = alpha (x) (A (x) B)) the pair determines P
 * exactly, and the form is unique.
 *
 * Pointers.  Every matrix / vector argument is a DEVICE pointer unless its
 * name ends in _host.  All buffers are owned by the caller; the library
 * keeps no pointer after a call returns.  Workspaces are sized with the
 * matching *_workspace_size call and passed in; the compute entry points
 * allocate no device memory.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Calls are stream-ordered and asynchronous unless documented as
 * synchronous.
 *
 * Errors.  Argument errors are returned synchronously.  Data-dependent
 * errors (a finite value above MPR_FMAX that would enter a product) are
 * reported on the device: *d_status (a device int32 the caller zeroes) is
 * set to MPR_EOVERFLOW, and the results of that call are then unspecified.
 * A wrong answer is never produced silently: either *d_status stays 0 or
 * the call's outputs must be discarded.
 */
#ifndef MPR_H
#define MPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPR_OK = 0,
    MPR_EINVAL = 1,       /* bad argument (size, pointer, leading dimension) */
    MPR_ENOMEM = 2,       /* workspace too small */
    MPR_EOVERFLOW = 3,    /* finite value above MPR_FMAX would enter a product */
    MPR_ENOTFOUND = 4,    /* no periodic regime up to the requested power */
    MPR_EHIP = 5,         /* HIP runtime error */
    MPR_EUNSUPPORTED = 6, /* no gfx950 device, or a size beyond the limits */
    MPR_ETIMEDOUT = 7,    /* query server: the request waited past its deadline */
    MPR_ECANCELED = 8     /* query server: the request was cancelled */
} mpr_status;

#define MPR_INF 0xFFFFu
#define MPR_FMAX 0x7FFFu
#define MPR_ROW_NONE INT64_MAX
#define MPR_CHAIN 0  /* A^e = (((A (x) A) (x) A) ...): e-1 products */
#define MPR_SQUARE 1 /* binary powering: squares A^(2^j) and their products */
#define MPR_CHAIN_SPARSE 2 /* the chain, each step over only the rows of A that
                            * reach each block of output columns */
#define MPR_PERIOD_SPARSE 1 /* mpr_find_period_ex flag: compressed-K chain steps */
#define MPR_PERIOD_EXTEND 2 /* mpr_find_period_ex flag: stop at the confirmed
                               period and extend the traces by it */
#define MPR_PERIOD_REUSE_A 4 /* mpr_find_period_ex flag: A's buffer may be
                                overwritten to hold a power (needs
                                MPR_PERIOD_SPARSE) */
#define MPR_PERIOD_PIPELINE 8 /* mpr_find_period_ex flag: compute the next
                                 power while the host reads the current
                                 one's class hash (not with
                                 MPR_PERIOD_REUSE_A) */

/* Arithmetic of a product configuration.  MPR_ARITH_U16: packed uint16
 * saturating add and min.  MPR_ARITH_F16: the operands' f16 images (a
 * finite value below 0x800 is its own f16 bit pattern, 0xFFFF is +inf,
 * larger finite values are clamped to 0x800), two k per packed 3-input
 * minimum; round-to-nearest is exact below 2048, so every result below
 * 0x800 or infinite is exact, and a tile holding any other result is
 * recomputed in uint16.  Both give the same C bit for bit. */
#define MPR_ARITH_U16 0
#define MPR_ARITH_F16 1

typedef void *mpr_stream;

/* Library version (major*10000 + minor*100 + patch). */
int mpr_version(void);
/* Static string naming a status code. */
const char *mpr_status_string(int status);
/* Checks that device `device` is a gfx950 part and records its CU count.
 * Synchronous.  Called implicitly by every entry point on first use. */
mpr_status mpr_init(int device);

/* ------------------------------------------------------------------ */
/* Transfer matrix (Section 4.1, Definition 4, Corollary 7).           */
/* ------------------------------------------------------------------ */

/* Number of correct words of length m (Definition 4; Table 1 lists them):
 * words over {a,b,c,d} with none of ad, da, ab, ba, bb as neighbours.
 * 1 <= m <= 12.  Synchronous, host only. */
mpr_status mpr_transfer_size(int m, int64_t *n_states_host);

/* The correct words in state order (increasing base-4 value, row 1 the most
 * significant letter; a=0, b=1, c=2, d=3), m bytes per word, into the host
 * buffer words_host of capacity_words words.  Synchronous, host only. */
mpr_status mpr_transfer_words(int m, uint8_t *words_host, int64_t capacity_words);

/* Writes A(G) of Corollary 7 into the device matrix A (n x n, n from
 * mpr_transfer_size, row stride lda >= n): A[q][p] = 2 p(a) + p(b) when
 * word p can follow word q under the rule lists of Section 4.1 (row q is
 * the previous column, p the next), else MPR_INF.  1 <= m <= 11. */
mpr_status mpr_build_transfer(int m, uint16_t *A, int64_t lda, mpr_stream stream);

/* Border ("loss") matrix of the appendix (proof of Lemma 10) for a strip
 * of m rows: same states; rows 1..m-1 follow the rule lists above, and the
 * m-th row need not be dominated (after q_m = d every label allowed after
 * q_m = c is allowed).  Arc label 10 p(a) + 5 p(b) - 2 nd(q, p), with nd the
 * newly dominated vertices of Algorithm 3, so a closed walk of n arcs weighs
 * 5 g - 2 |D(g)| = 2 L_a of the almost Roman dominating function g it
 * encodes.  Labels can be negative, so every finite entry is written plus
 * *shift_host = 2 (3m + 1) (host output): traces of the n-th power exceed
 * 2 L_a(n) by n * shift, and a period (mu, lam, c') found on this matrix has
 * c = c' - lam * shift.  Device matrix n x n (lda), 1 <= m <= 11. */
mpr_status mpr_build_border_transfer(int m, uint16_t *A, int64_t lda, int64_t *shift_host, mpr_stream stream);

/* ------------------------------------------------------------------ */
/* (min,+) products (Section 3).                                       */
/* ------------------------------------------------------------------ */

/* C = A (x) B: C[i][j] = min_k sat(A[i][k] + B[k][j]) with A M x K (lda),
 * B K x N (ldb), C M x N (ldc).  Exact for inputs whose finite entries are
 * <= MPR_FMAX; when d_status != NULL the inputs are checked first and
 * *d_status is set to MPR_EOVERFLOW if one is not (pass NULL only when the
 * caller guarantees the bound).  Finite outputs are exact values in
 * [0, 0xFFFE].  M, N, K >= 0 (an empty K gives an all-MPR_INF C).  C must
 * not overlap A or B.  Fast path: A, B, C 16-byte aligned and lda, ldb, ldc
 * multiples of 8; any other layout takes a slower element-wise path.  The
 * configuration comes from the tile table of the process-wide arithmetic
 * (mpr_set_arith): packed uint16 by default; in the f16 form the result is
 * the same, but tiles whose minima reach 2048 are computed twice (about
 * 1.75x the uint16 time for such tiles). */
mpr_status mpr_minplus_gemm(int64_t M, int64_t N, int64_t K,
                            const uint16_t *A, int64_t lda,
                            const uint16_t *B, int64_t ldb,
                            uint16_t *C, int64_t ldc,
                            int32_t *d_status, mpr_stream stream);

/* Same with an explicit tile configuration (0 <= cfg < mpr_gemm_config_count);
 * used by the autotuner.  cfg = -1 picks from the tile table. */
mpr_status mpr_minplus_gemm_cfg(int cfg, int64_t M, int64_t N, int64_t K,
                                const uint16_t *A, int64_t lda,
                                const uint16_t *B, int64_t ldb,
                                uint16_t *C, int64_t ldc,
                                int32_t *d_status, mpr_stream stream);

/* The same product (same bits) launched so that each CU holds one
 * workgroup of it fewer than it could: every workgroup reserves extra LDS,
 * so the registers of one workgroup slot per CU stay free for the waves of
 * other launches for as long as the product runs (without it a long
 * product holds every slot until its blocks retire, milliseconds each).  A
 * configuration that fits fewer than 3 workgroups per CU runs as the
 * 128 x 128 tile of the same arithmetic.  Costs well under 1 % at the sizes
 * measured (N = 7411 to 21909).  For callers that run long products beside
 * latency-sensitive work: the query server builds its large ladders with
 * it.  cfg = -1 picks from the tile table.  Arguments and errors as
 * mpr_minplus_gemm. */
mpr_status mpr_minplus_gemm_spare(int cfg, int64_t M, int64_t N, int64_t K,
                                  const uint16_t *A, int64_t lda,
                                  const uint16_t *B, int64_t ldb,
                                  uint16_t *C, int64_t ldc,
                                  int32_t *d_status, mpr_stream stream);

/* Row-min normalisation in place: for each row i of the M x N matrix C,
 * r_i = least finite entry, C[i][:] -= r_i (MPR_INF stays), and
 * R_out[i] = R_in[i] + r_i (R_in may be NULL, read as 0; R_in may equal
 * R_out).  An all-infinite row, or R_in[i] == MPR_ROW_NONE, gives
 * R_out[i] = MPR_ROW_NONE.  *d_status = MPR_EOVERFLOW when a normalised
 * finite entry exceeds MPR_FMAX (the result can not enter a product). */
mpr_status mpr_normalise(int64_t M, int64_t N, uint16_t *C, int64_t ldc,
                         const int64_t *R_in, int64_t *R_out,
                         int32_t *d_status, mpr_stream stream);

/* Workspace bytes for mpr_minplus_gemm_norm with a K x N right operand. */
mpr_status mpr_gemm_norm_workspace_size(int64_t K, int64_t N, size_t *bytes_host);

/* Canonical product of two canonical forms:
 * (Rc, C) = canon((Ra (+) A) (x) (Rb (+) B)).  With s = min_l Rb[l], the
 * right operand is folded to B'[l][j] = B[l][j] + (Rb[l] - s) (scalar rule
 * of Section 3) in the workspace, then C = canon(A (x) B') and
 * Rc = Ra + s + rowmin.  Ra / Rb may be NULL (all zero).  A is M x K, B is
 * K x N, C is M x N.  *d_status = MPR_EOVERFLOW when a folded entry or a
 * normalised output exceeds MPR_FMAX. */
mpr_status mpr_minplus_gemm_norm(int64_t M, int64_t N, int64_t K,
                                 const uint16_t *A, int64_t lda, const int64_t *Ra,
                                 const uint16_t *B, int64_t ldb, const int64_t *Rb,
                                 uint16_t *C, int64_t ldc, int64_t *Rc,
                                 void *ws, size_t ws_bytes,
                                 int32_t *d_status, mpr_stream stream);

/* ------------------------------------------------------------------ */
/* Powers (Algorithm 1, step 3; Algorithm 2, step 3).                  */
/* ------------------------------------------------------------------ */

/* Workspace bytes for mpr_minplus_power on an n x n matrix.  For
 * MPR_CHAIN on a matrix too small to fill the device (fewer than about
 * two 64 x 64 output tiles per CU) this includes the partial products of
 * steps whose inner dimension is split into ranges (the minimum over k
 * taken in parts, then the minimum of the parts: the same bits); a
 * workspace of only the layout, n * round_up(n, 8) * 2 + 256 bytes, runs
 * every step unsplit. */
mpr_status mpr_power_workspace_size(int64_t n, int64_t e, int schedule, size_t *bytes_host);

/* Canonical form (N_out, R_out) of A^e for the n x n matrix A, e >= 1.
 * schedule = MPR_CHAIN computes A^k = A^(k-1) (x) A with A kept raw and a
 * normalisation after every product (e-1 products); MPR_SQUARE uses binary
 * powering on canonical forms; MPR_CHAIN_SPARSE is the chain with each step
 * restricted, per block of 64 output columns J, to the rows L_J of A that
 * have a finite entry in J (C[:, J] = N[:, L_J] (x) A[L_J, J], the same
 * product; worth it when A is sparse, as transfer matrices are).  All three
 * give identical bits.  N_out is n x n
 * (ldo), R_out has n entries.  For MPR_CHAIN_SPARSE a workspace smaller
 * than mpr_power_workspace_size gives the plan what is left after the
 * chain buffer (see mpr_sparse_plan_bytes); d_status must then be given. */
mpr_status mpr_minplus_power(const uint16_t *A, int64_t n, int64_t lda, int64_t e,
                             int schedule, uint16_t *N_out, int64_t ldo, int64_t *R_out,
                             void *ws, size_t ws_bytes, int32_t *d_status, mpr_stream stream);

/* Resumes a chain (Algorithm 2's step A^(k+1) = A^k (x) A, kept in
 * canonical form as mpr_minplus_power does) from a power saved earlier:
 * given (N_k, R_k), the canonical form of A^k (N_k n x n, row stride ldk,
 * entries <= MPR_FMAX, e.g. copied back from a checkpoint on the host),
 * writes the canonical form of A^(k + steps) to (N_out, R_out) by `steps`
 * steps of the chain (schedule MPR_CHAIN or MPR_CHAIN_SPARSE), the same
 * bits as mpr_minplus_power(A, k + steps) would give: row i of a power
 * depends only on row i of the previous one and on A, so the state of a
 * chain is (N_k, R_k, k).  steps = 0 copies.  N_out may be N_k (then
 * ldo == ldk) and R_out may be R_k.  Workspace:
 * mpr_power_workspace_size(n, steps + 1, schedule) bytes (for
 * MPR_CHAIN_SPARSE the plan rules of mpr_minplus_power apply).  N_k is
 * checked like A (d_status). */
mpr_status mpr_chain_resume(const uint16_t *A, int64_t n, int64_t lda,
                            const uint16_t *N_k, int64_t ldk, const int64_t *R_k,
                            int64_t steps, int schedule, uint16_t *N_out, int64_t ldo,
                            int64_t *R_out, void *ws, size_t ws_bytes,
                            int32_t *d_status, mpr_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as mpr_minplus_power, with its workspace taken from a fixed
 * device array of MPR_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends (its address on each device is
 * recorded by mpr_init / the first call there).  The caller still passes A,
 * N_out, R_out and d_status (same meaning, layout and errors as
 * mpr_minplus_power).  Returns MPR_ENOMEM, before launching anything, when
 * mpr_power_workspace_size(n, e, schedule) exceeds the array (for example
 * n > 5792 for MPR_CHAIN); allocates nothing and calls no allocating
 * routine.  The array keeps the last call's contents (nothing in it needs
 * clearing: every call writes what it reads).  All calls on one GPU share
 * the array, so calls that overlap on that GPU (other streams, other host
 * threads) race and give unspecified results: serialise them. */
#define MPR_NOALLOC_SCRATCH_BYTES (64u << 20)
mpr_status mpr_minplus_power_noalloc(const uint16_t *A, int64_t n, int64_t lda, int64_t e, int schedule,
                                     uint16_t *N_out, int64_t ldo, int64_t *R_out, int32_t *d_status,
                                     mpr_stream stream);

/* Bytes of the compressed-K plan of the n x n device matrix A (row stride
 * lda): for every block J of 64 columns, the rows of A with a finite entry
 * in J (rounded up to 32 per block) and their packed entries -- a few per
 * cent of the worst case that mpr_power_workspace_size and
 * mpr_period_workspace_size_ex assume (a dense A) for transfer matrices.
 * A workspace of mpr_power_workspace_size(n, e, MPR_CHAIN) + this many bytes
 * serves mpr_minplus_power(..., MPR_CHAIN_SPARSE) on this A (a d_status is
 * then required: a plan that does not fit its share sets MPR_ENOMEM there
 * and the call computes nothing), and mpr_period_workspace_size_ex(n,
 * slots, 0) + this many bytes serves mpr_find_period_ex with
 * MPR_PERIOD_SPARSE (which sizes the plan itself and gives the ring every
 * other byte).  SYNCHRONOUS on stream; sizing only: it allocates and frees a
 * device temporary of about 16 (n / 64 + 2) bytes. */
mpr_status mpr_sparse_plan_bytes(const uint16_t *A, int64_t n, int64_t lda, size_t *bytes_host, mpr_stream stream);

/* Corollary 7: *d_gamma = min_i (R[i] + N[i][i]) over rows with a finite
 * diagonal entry (MPR_ROW_NONE if there is none).  For N, R = A^n this is
 * gamma_R(P_m x C_n), n >= 3. */
mpr_status mpr_trace_min(const uint16_t *N, int64_t n, int64_t ld, const int64_t *R,
                         int64_t *d_gamma, mpr_stream stream);

/* Trace of a product without forming it:
 * *d_gamma = min_i min_l (RX[i] + X[i][l] + RY[l] + Y[l][i]), i.e. the
 * trace of (RX (+) X) (x) (RY (+) Y).  RX / RY may be NULL (zero). */
mpr_status mpr_trace_of_product(const uint16_t *X, const int64_t *RX,
                                const uint16_t *Y, const int64_t *RY,
                                int64_t n, int64_t ld, int64_t *d_gamma, mpr_stream stream);

/* The same trace (Corollary 7) with the right operand given through the
 * canonical form of its transpose: Y[l][i] = CY[i] + YT[i][l], so
 * *d_gamma = min_i (RX[i] + CY[i] + min_l (X[i][l] + YT[i][l])) -- for
 * YT, CY = the canonical form of (A^T)^j = (A^j)^T this is the trace of
 * (RX (+) X) (x) A^j.  X and YT: device, n x n, row stride ld, any uint16
 * (0xFFFF = infinity, sums exact in 32 bits); RX / CY: device, n int64
 * each, MPR_ROW_NONE for an empty row, NULL for zero.  Both operands are
 * read along rows once (a streaming pass, no transpose).  *d_gamma is
 * MPR_ROW_NONE when every term has an infinite operand.  Asynchronous on
 * stream. */
mpr_status mpr_trace_of_product_t(const uint16_t *X, const int64_t *RX,
                                  const uint16_t *YT, const int64_t *CY,
                                  int64_t n, int64_t ld, int64_t *d_gamma, mpr_stream stream);

/* ------------------------------------------------------------------ */
/* Periodic regime (Lemma 2, Proposition 8, Algorithm 2).              */
/* ------------------------------------------------------------------ */

/* Workspace bytes to keep `slots` powers of an n x n matrix resident
 * (slots >= 2).  The period search keeps the last `slots` powers in a ring,
 * so it can confirm a period lam only when lam < slots; mu is unbounded.
 * The ring takes every byte of the workspace past the fixed part (and, with
 * MPR_PERIOD_SPARSE, past the plan, sized for the given A). */
mpr_status mpr_period_workspace_size(int64_t n, int64_t slots, size_t *bytes_host);

/* Least (mu, lam, c) with A^(mu+lam) = c (x) A^mu, searching the chain
 * A^1 .. A^kmax.  The classes of A^k up to a scalar shift form an
 * eventually periodic sequence; the first repeated class (found by a
 * 64-bit class hash, then confirmed by an exact compare of (N, R - R'))
 * gives the least pre-period mu and the least period lam (confirmable when
 * lam is smaller than the number of power slots the workspace holds; the
 * class hashes of all earlier powers stay on the host).  When traces_host
 * is not NULL it receives kmax + 1 int64 values, traces_host[k] = trace of
 * A^k for k = 1..kmax (the chain then always runs to kmax), else the search
 * stops at the first confirmed repeat.  When A^mu has no finite entry
 * (a nilpotent A) every c fits and *c_host = 0.  SYNCHRONOUS on `stream`.
 * Returns MPR_ENOTFOUND when no repeat is confirmed (also when no periodic
 * regime exists, e.g. components of A with different mean cycle weights),
 * MPR_EOVERFLOW on overflow. */
mpr_status mpr_find_period(const uint16_t *A, int64_t n, int64_t lda, int64_t kmax,
                           int64_t *mu_host, int64_t *lam_host, int64_t *c_host,
                           int64_t *traces_host, void *ws, size_t ws_bytes, mpr_stream stream);

/* Installs a process-wide observer of the period search: fn(k, trace, user)
 * is called on the searching thread after every power A^k it computes
 * (trace = its trace, MPR_ROW_NONE if none), e.g. to report progress of a
 * search that runs for minutes.  fn = NULL removes it. */
mpr_status mpr_set_period_progress(void (*fn)(int64_t k, int64_t trace, void *user), void *user);

/* Proposition 8 and the finite-difference solution that follows it: with
 * A^(mu+lam) = c (x) A^mu, gamma(n + lam) = gamma(n) + c for n >= mu, so
 *   gamma(n) = traces[mu + (n - mu) mod lam] + c * floor((n - mu) / lam)
 * for n >= mu, and traces[n] below mu.  traces_host[k] (k <= kmax) are the
 * traces of A^k as mpr_find_period returns them; needs mu + lam - 1 <= kmax
 * (and n <= kmax when n < mu).  A residue class whose trace is MPR_ROW_NONE
 * (no closed walk of that length) gives MPR_ROW_NONE for every n in it.
 * Host only. */
mpr_status mpr_gamma_from_period(int64_t mu, int64_t lam, int64_t c, const int64_t *traces_host,
                                 int64_t kmax, int64_t n, int64_t *gamma_host);
/* The same solution as a closed form: for n >= mu,
 *   gamma(n) = (c * n + numer_host[n mod lam]) / lam   (an exact division),
 * numer_host receiving lam int64 values; numer_host[r] = MPR_ROW_NONE when
 * residue class r has no finite trace.  Host only. */
mpr_status mpr_period_formula(int64_t mu, int64_t lam, int64_t c, const int64_t *traces_host,
                              int64_t kmax, int64_t *numer_host);

/* mpr_find_period with flags: MPR_PERIOD_SPARSE runs the chain steps as
 * MPR_CHAIN_SPARSE does (identical results).  The workspace must then be
 * sized by mpr_period_workspace_size_ex with the same flags (the worst
 * case), or by mpr_period_workspace_size_ex(n, slots, 0) plus
 * mpr_sparse_plan_bytes of this A.
 * MPR_PERIOD_EXTEND stops at the power that confirms the period (k = mu +
 * lambda, as Algorithm 2 does) instead of computing every power to kmax,
 * and fills traces_host[k] for mu + lambda < k <= kmax from the relation
 * A^(k) = c (x) A^(k - lambda), k - lambda >= mu (Lemma 2):
 * trace(k) = trace(k - lambda) + c, exact (MPR_ROW_NONE stays).
 * MPR_PERIOD_REUSE_A (with MPR_PERIOD_SPARSE; lda must be round_up(n, 8))
 * is for matrices too large for a ring longer than the period: once the
 * compressed-K plan has replaced A, A's buffer (whose contents are then
 * lost) keeps the power at which a class repeat the ring can no longer
 * confirm was seen, and the repeat is confirmed exactly one period later.
 * *mu_host is then that power's index, the smallest power at which the
 * relation A^(mu+lam) = c (x) A^mu has been checked exactly (at most lam
 * above the least pre-period, which the class hashes place lam below it);
 * lam and c are the least period and its exact offset.
 * MPR_PERIOD_PIPELINE enqueues power k + 1 before the host waits for the
 * class hash, trace and status of power k (read through pinned host
 * memory, allocated and freed by the call), so the host round trip of each
 * power overlaps the next one's work instead of following it (it matters
 * where a power takes tens of microseconds: small matrices).  Same
 * results.  The power computed ahead takes a ring buffer, which
 * mpr_period_workspace_size_ex counts with this flag: a workspace of
 * `slots` ring powers still confirms periods up to slots - 1.  The call
 * synchronises the stream before it returns. */
mpr_status mpr_period_workspace_size_ex(int64_t n, int64_t slots, int flags, size_t *bytes_host);
mpr_status mpr_find_period_ex(const uint16_t *A, int64_t n, int64_t lda, int64_t kmax, int flags,
                              int64_t *mu_host, int64_t *lam_host, int64_t *c_host, int64_t *traces_host,
                              void *ws, size_t ws_bytes, mpr_stream stream);

/* ------------------------------------------------------------------ */
/* Batched power chains: one launch.                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint16_t *A; /* device, n x n, row stride lda; finite entries <= MPR_FMAX */
    int64_t n;
    int64_t lda;
    int64_t e;         /* exponent >= 1; computed by the chain schedule */
    uint16_t *N_out;   /* device, n x n, row stride ldo */
    int64_t ldo;
    int64_t *R_out;    /* device, n entries */
} mpr_chain_desc;

/* Workspace bytes for a batch described by the HOST array descs_host. */
mpr_status mpr_batch_workspace_size(const mpr_chain_desc *descs_host, int count, size_t *bytes_host);

/* Plans a batch into the workspace: splits every chain into row panels
 * (row i of A^k depends only on row i of A^(k-1) and on A, so panels never
 * wait on each other), orders the panels longest first (a ragged last
 * panel costs as much as a full one) and uploads the work list.
 * Synchronous.  MPR_EUNSUPPORTED beyond 2^31 - 1 panels.  The workspace
 * then holds the whole launch state; mpr_batch_launch may be called (or
 * captured) any number of times. */
mpr_status mpr_batch_plan(const mpr_chain_desc *descs_host, int count,
                          void *ws, size_t ws_bytes, mpr_stream stream);

/* Runs a planned batch: resets the work counter with a fill kernel and
 * launches the batch kernel, whose workgroups take the panels longest first
 * with one atomic add each (one workgroup per panel, or a persistent grid;
 * mpr_set_batch_persistent).  No memset node, no host sync, so the pair can
 * be captured into a HIP graph.  Results land in each N_out / R_out. */
mpr_status mpr_batch_launch(void *ws, int32_t *d_status, mpr_stream stream);

/* Describes the plan held in ws: configuration, workgroups of the grid
 * (one per panel, or the resident workgroups in the persistent form) and
 * number of panels (host ints, any may be NULL).  MPR_EINVAL if ws holds no
 * plan. */
mpr_status mpr_batch_plan_info(void *ws, int *cfg, int *grid, int *panels);

/* Launch form of the plans made after the call (process-wide): 0 (the
 * default) one workgroup per panel, 1 a persistent grid of the resident
 * workgroups, each looping over the work list until it is empty.  Same
 * results; the per-panel form is faster on MI355X because the CU's wave
 * arbiter favours older waves.  MPR_EINVAL for other values. */
mpr_status mpr_set_batch_persistent(int on);

/* Plan + launch. */
mpr_status mpr_batch_power(const mpr_chain_desc *descs_host, int count,
                           void *ws, size_t ws_bytes, int32_t *d_status, mpr_stream stream);

/* Arithmetic (MPR_ARITH_*) of the compressed-K chain steps of
 * MPR_CHAIN_SPARSE and MPR_PERIOD_SPARSE; MPR_ARITH_U16 by default (and
 * whatever mpr_set_arith last set).  Both give the same powers bit for
 * bit.  Process-wide setting. */
mpr_status mpr_set_sparse_arith(int arith);

/* Form of the compressed-K chain steps (Algorithm 2's step restricted to
 * the rows L_J of A that reach each block J of 64 output columns):
 * MPR_SPARSE_TILES multiplies N[:, L_J] by the dense rows A[L_J, J];
 * MPR_SPARSE_ENTRIES (uint16 arithmetic only; the f16 form always takes
 * the tiles) visits only the finite entries of A[L_J, J], one output
 * column per wave; MPR_SPARSE_AUTO (the default) picks by the matrix's
 * size.  Both give the same powers bit for bit.  MPR_EINVAL for other
 * values.  Process-wide setting. */
#define MPR_SPARSE_AUTO 0
#define MPR_SPARSE_TILES 1
#define MPR_SPARSE_ENTRIES 2
mpr_status mpr_set_sparse_form(int form);

/* Process-wide arithmetic (MPR_ARITH_U16, the default, or MPR_ARITH_F16) of
 * every product whose configuration the library picks: products with
 * cfg = -1 (the tile table of that arithmetic), the steps of
 * mpr_minplus_power, mpr_find_period and the server's ladder builds, the
 * compressed-K steps (as mpr_set_sparse_arith) and the configuration that
 * mpr_batch_plan chooses.  Results are identical bit for bit in both;
 * MPR_EINVAL for other values.  Calls already enqueued keep the arithmetic
 * they were launched with. */
mpr_status mpr_set_arith(int arith);
/* The current process-wide arithmetic (MPR_ARITH_*). */
int mpr_get_arith(void);

/* Number of compiled batched-kernel configurations (panel heights). */
int mpr_batch_config_count(void);
/* Rows per panel, threads per workgroup and arithmetic (MPR_ARITH_*) of
 * batched configuration cfg (host ints, any may be NULL). */
mpr_status mpr_batch_config_info(int cfg, int *panel_rows, int *threads, int *arith);
/* Forces the configuration later mpr_batch_plan calls use (-1 = choose by
 * a longest-first schedule model of the batch among the configurations of
 * the process-wide arithmetic).  Process-wide setting. */
mpr_status mpr_set_batch_config(int cfg);
/* Relative throughputs the schedule model weighs each batched
 * configuration by (count = mpr_batch_config_count(); rel_host[c] > 0, or
 * 0 to exclude configuration c; each arithmetic must keep one).  The batch
 * autotuner measures them; rel_host = NULL restores the compiled-in
 * values.  Process-wide; MPR_EINVAL on a bad count or value. */
mpr_status mpr_set_batch_weights(const double *rel_host, int count);
/* Copies the weights in use into rel_host (capacity count). */
mpr_status mpr_get_batch_weights(double *rel_host, int count);

/* Captures mpr_batch_launch(ws, d_status) on `stream` into an instantiated
 * HIP graph returned in *graph_host (opaque).  Synchronous. */
mpr_status mpr_batch_graph_create(void *ws, int32_t *d_status, mpr_stream stream, void **graph_host);
/* Replays a captured graph on `stream`. */
mpr_status mpr_graph_launch(void *graph, mpr_stream stream);
/* Destroys a captured graph. */
mpr_status mpr_graph_destroy(void *graph);

/* ------------------------------------------------------------------ */
/* Query server: continuous batching of gamma_R(P_m x C_n) requests.   */
/* ------------------------------------------------------------------ */

typedef struct {
    int device;               /* HIP device the engine runs on */
    int baby;                 /* B: baby steps A^1..A^B, giant steps A^(B i) */
    int64_t max_n;            /* largest n served (n >= 3) */
    int max_batch;            /* most queries in one grouped launch */
    int slots;                /* grouped launches in flight (1..64), plus one
                                 on a stream of its own for queries of
                                 ladders still being built */
    size_t hbm_budget_bytes;  /* ladders are admitted only within this */
    int wide_only;            /* 0: keep byte copies of the ladder powers and
                                 answer from them when every finite entry is
                                 <= 127 (half the bytes per query; exact);
                                 1: uint16 only */
    int busy_poll;            /* 1: the worker thread never sleeps (one CPU core
                                 busy; a request is picked up without a thread
                                 wake-up); 0: it sleeps until a request or a
                                 launch needs it */
    int period_mode;          /* 0: the per-query GPU path above.  1: the
                                 labelled fast mode of Proposition 8: the
                                 build of m searches the period of A
                                 (compressed-K steps, 8 ring powers, up to
                                 max_n) on its own host thread and stream,
                                 keeps the traces of A^1..A^max_n on the host
                                 (past the confirmed period, filled from it;
                                 all computed when no period shows up to
                                 max_n) and frees its device memory; a query
                                 is a table read with no GPU work.  baby,
                                 wide_only, max_batch and slots are unused. */
    double request_timeout_s; /* > 0: a request not yet launched this many
                                 seconds after its submission (waiting for
                                 its ladder, for memory or for a launch slot)
                                 is completed with MPR_ETIMEDOUT; 0: none */
} mpr_server_options;

typedef struct {
    int64_t tag;              /* the caller's tag from mpr_server_submit */
    int m;
    int64_t n;
    int64_t gamma;            /* gamma_R(P_m x C_n) when status == MPR_OK */
    int status;
    int cold;                 /* 1 when the request waited for a ladder build */
    double t_submit_s, t_start_s, t_done_s; /* server clock (mpr_server_now) */
} mpr_query_result;

typedef struct {
    int64_t submitted, completed, batches, max_batch_seen;
    int64_t builds, evictions, admission_waits, resident_bytes;
    int64_t narrow_builds;    /* finished builds whose queries read byte copies */
    int64_t shared_reads;     /* queries answered without a read of their own of
                                 the giant power: another query of the same
                                 launch with the same m and i read it for both
                                 (byte copies; groups of up to 8) */
    int64_t period_answers;   /* queries answered from a period table
                                 (period_mode) */
    int64_t early_answers;    /* queries answered from a ladder still being
                                 built (its giants up to theirs written) */
} mpr_server_stats;

/* Starts an engine with its own worker thread and two non-blocking HIP
 * streams (queries, ladder builds).  For each m it keeps the canonical
 * powers A^(B i), i <= (max_n - 1) / B, and the canonical forms of
 * (A^T)^j = (A^j)^T, j = 1..B, resident, and answers n = B i + j
 * (1 <= j <= B) as the trace of A^(B i) (x) A^j (Corollary 7) without
 * forming the product: one pass reading both matrices along rows (as
 * mpr_trace_of_product_t), over byte copies of them unless wide_only is set
 * or an entry does not fit (canonical Roman powers have entries <= 2m).
 * Queries of one launch on byte copies that share the giant power (same m
 * and i) are answered in groups of up to 8 that stream it once.  The engine allocates its ladders itself,
 * within hbm_budget_bytes (least recently used idle ladders are evicted;
 * requests that do not fit wait).  *server_host receives an opaque handle. */
mpr_status mpr_server_create(const mpr_server_options *opt, void **server_host);
/* Queues gamma_R(P_m x C_n); non-blocking and thread-safe.  Requests with
 * m outside 1..11 or n outside 3..max_n complete with MPR_EINVAL, those whose
 * ladder is larger than the whole budget with MPR_ENOMEM; a ladder whose
 * build fails completes its requests with the build's status. */
mpr_status mpr_server_submit(void *server, int m, int64_t n, int64_t tag);
/* Completes with MPR_ECANCELED every request with this tag that is still
 * waiting (not yet in a launch) when the worker next looks; a request
 * already launched or answered is not affected (its result comes as
 * usual).  Asynchronous: the outcome arrives through mpr_server_poll. */
mpr_status mpr_server_cancel(void *server, int64_t tag);
/* Moves up to capacity finished requests into out_host (host array),
 * waiting up to wait_ms for the first one.  *count_host = number moved. */
mpr_status mpr_server_poll(void *server, mpr_query_result *out_host, int capacity, int *count_host,
                           int wait_ms);
/* Counters of the engine (host struct). */
mpr_status mpr_server_stats_get(void *server, mpr_server_stats *out_host);
/* Seconds since the engine started, on the clock of the result times. */
double mpr_server_now(void *server);
/* Device bytes one ladder of m takes for the given baby step, max_n and
 * wide_only option. */
int64_t mpr_server_ladder_bytes(int m, int baby, int64_t max_n, int wide_only);
/* Device bytes a period-mode build of m holds while it runs (A and the
 * period search's workspace; none once the build ends); -1 for m outside
 * 1..11. */
int64_t mpr_server_period_bytes(int m);
/* Stops the worker, waits for outstanding GPU work, frees everything. */
mpr_status mpr_server_destroy(void *server);

/* ------------------------------------------------------------------ */
/* Tile configurations and the autotuner's table.                      */
/* ------------------------------------------------------------------ */

/* Measures the issue rate of a product's instruction mix on the current
 * device (MPR_ARITH_U16: v_pk_add_u16 clamp + v_pk_min_u16; MPR_ARITH_F16:
 * 2 v_pk_add_f16 + 1 v_pk_minimum3_f16): a register-only kernel with 8
 * waves per SIMD on every CU, each lane running independent accumulator
 * chains `iters` times (1 <= iters <= 2^24).  *pairs_per_s_host receives the
 * (add, min) pairs per second by HIP events; *clock_ghz_host the shader
 * clock during the run, from the cycle counter and the constant-rate wall
 * clock of one wave.  Confirms the VALU peak the kernels are priced
 * against.  Synchronous; allocates (and frees) 256 bytes of device memory,
 * so not for a hot path. */
mpr_status mpr_valu_probe(int arith, int iters, double *pairs_per_s_host, double *clock_ghz_host,
                          mpr_stream stream);

/* Number of compiled (min,+) tile configurations. */
int mpr_gemm_config_count(void);
/* Describes configuration cfg: tile rows, columns, k depth, per-lane
 * rows/columns, threads per workgroup and arithmetic (MPR_ARITH_*) (host
 * ints, any may be NULL). */
mpr_status mpr_gemm_config_info(int cfg, int *bm, int *bn, int *bk, int *tm, int *tn, int *threads,
                                int *arith);
/* The configuration the tile table of the process-wide arithmetic gives an
 * M x N x K product (cfg = -1). */
int mpr_gemm_pick_config(int64_t M, int64_t N, int64_t K);
/* Installs a size -> configuration table used when cfg = -1: entry t
 * applies to problems whose largest dimension is <= max_dim_host[t]
 * (ascending); larger problems use the last entry.  Every entry must name
 * a configuration of one arithmetic, and the table replaces that
 * arithmetic's table (products use the table of the process-wide
 * arithmetic, mpr_set_arith).  Copies the arrays. */
mpr_status mpr_set_tile_table(const int64_t *max_dim_host, const int *cfg_host, int entries);
/* Times every configuration on an n x n x n product (random operands made
 * inside; allocates, so not for use on a hot path) and writes the average
 * milliseconds per product into ms_host[cfg]; returns the fastest in
 * *best_host.  Synchronous. */
mpr_status mpr_autotune_gemm(int64_t n, int reps, float *ms_host, int *best_host, mpr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* MPR_H */
