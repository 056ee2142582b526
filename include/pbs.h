/*
 * pbs.h -- C ABI of the Pauli-sum operator-state library for AMD MI355X (gfx950).
 *
 * Implements the data-parallel path of "A High-Performance Pauli-Algebra
 * Framework for Large-Scale Quantum Simulations" (arXiv 2606.28952): Pauli
 * strings in binary symplectic form (Section 2.2), their products and
 * canonical linear combinations (Section 2.3), the Jordan-Wigner Hamiltonian
 * built directly from integrals (Section 2.3, Algorithm 1), grouping by
 * X-mask (Section 2.4, Eq. topological_group), the full and spin-sector
 * configuration spaces (Section 2.4, spin-resolved product basis; Eq. fcidim)
 * and the target-driven operator-state product (Eq. reverse_sum,
 * Eq. sreverse_sum) with the energy of Eq. vqe_energy.  Every data-parallel
 * step runs as a HIP kernel on the caller's stream.
 *
 * Conventions used throughout
 * ---------------------------
 *  - Qubit k is bit k of a basis index (Eqs. xp_encoding, zp_encoding).  A
 *    mask of n qubits occupies W = ceil(n/64) uint64 words, word w holding
 *    qubits 64w..64w+63; arrays of strings are term-major: x[i*W + w].
 *  - A string (x, z, g) in "letter form" is i^g times the tensor product of
 *    sigma^(x_k, z_k) with (0,0)=I, (1,0)=X, (1,1)=Y, (0,1)=Z
 *    (Eq. single_pauli_mapping, Eq. pauli_group); g is a Z4 exponent stored
 *    in a uint8 (values 0..3).  Pauli-sum coefficients at this boundary are in
 *    letter form, complex float64 stored as interleaved (re, im) doubles, so a
 *    Hermitian sum has real coefficients.  Kernels use the XZ form
 *    C_k = c_k * i^popcount(x_k & z_k) internally (Section 2.3).
 *  - Canonical form (Section 2.3): unique strings sorted by (X, Z) read as
 *    unsigned big integers, X major; every coefficient is the correctly
 *    rounded (nearest-even) exact sum of its contributions, real and
 *    imaginary parts separately, with exact zeros written as +0.0; a term is
 *    dropped when max(|Re c|, |Im c|) <= eps_drop (pass a negative eps_drop
 *    to keep exact zeros).
 *  - Sector spaces use n_orb spatial orbitals on 2*n_orb qubits: qubits
 *    0..n_orb-1 hold the alpha string, n_orb..2n_orb-1 the beta string.  Spin
 *    strings are enumerated in ascending integer order and a configuration's
 *    index is rank_alpha * D_beta + rank_beta.
 *  - State vectors are complex, interleaved (re, im), either complex128
 *    (PBS_C128) or complex64 (PBS_C64); all accumulation is float64.
 *
 * Memory and streams
 * ------------------
 *  - Handles (pbs_sum, pbs_grouped, pbs_space) own device memory; it is
 *    allocated when a handle is built and released by its destroy call.
 *    Handles are immutable after creation except through
 *    pbs_pauli_canonicalize, so concurrent const use is thread-safe.
 *  - Pointers documented as "device" must be device (or managed) memory on
 *    the current HIP device; pointers documented as "host or device" may be
 *    either.  State vectors, outputs and workspaces are owned by the caller.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls documented as
 *    asynchronous only enqueue work; calls that build handles synchronize the
 *    stream before returning.
 *
 * Errors
 * ------
 *  Every call returns a pbs_status; no exception crosses the ABI.  On error
 *  pbs_last_error() returns a message for the calling thread (valid until the
 *  thread's next call).  HIP failures map to PBS_ERR_DEVICE.
 */
#ifndef PBS_H_
#define PBS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pbs_status;
#define PBS_OK 0
#define PBS_ERR_ARG 1         /* null pointer, bad enum, inconsistent sizes, overlapping buffers */
#define PBS_ERR_RANGE 2       /* size or qubit count beyond what the call supports */
#define PBS_ERR_ALLOC 3       /* device or host allocation failed */
#define PBS_ERR_DEVICE 4      /* a HIP runtime call failed */
#define PBS_ERR_UNSUPPORTED 5 /* valid request outside the implemented cases */

typedef enum { PBS_C128 = 0, PBS_C64 = 1 } pbs_dtype;

typedef struct pbs_sum pbs_sum;         /* Pauli sum: strings + letter-form coefficients */
typedef struct pbs_grouped pbs_grouped; /* sum grouped by X-mask, kernel tables */
typedef struct pbs_space pbs_space;     /* configuration space (full or spin sector) */
typedef struct pbs_batch pbs_batch;     /* prepared launch of many operator-state products */
typedef struct pbs_vqe pbs_vqe;         /* Pauli-rotation ansatz with energy and gradient */
typedef struct pbs_mlp pbs_mlp;         /* warm-start network: parameters, optimizer state, buffers */

/* Message describing the calling thread's last failure ("" after success). */
const char* pbs_last_error(void);

/* Library ABI version (increments on any signature change). */
int32_t pbs_abi_version(void);

/* ------------------------------------------------------------------ strings */

/* Elementwise product of Pauli strings, out_i = A_i * B_i (Section 2.3,
 * Eqs. pauli_prod_x, pauli_prod_z, pauli_prod_phase): X and Z masks are
 * XORed and the Z4 phase is computed from popcounts.
 *  n_qubits  1..256; W = ceil(n_qubits/64) words per mask.
 *  n         number of string pairs.
 *  xa, za    device, n*W words each; pa device, n letter-form phases (0..3).
 *  xb, zb, pb  same for the right factors.
 *  xo, zo, po  device outputs; they may alias the inputs exactly.
 * Asynchronous.  Bits at or above n_qubits must be zero (not checked). */
pbs_status pbs_pauli_mul(uint32_t n_qubits, uint64_t n, const uint64_t* xa, const uint64_t* za, const uint8_t* pa,
                         const uint64_t* xb, const uint64_t* zb, const uint8_t* pb, uint64_t* xo, uint64_t* zo,
                         uint8_t* po, void* stream);

/* ------------------------------------------------------------------ Pauli sums */

/* Builds a sum handle from n_terms strings with letter-form coefficients
 * (arrays X, Z, C of Section 2.3).  x, z: host or device, n_terms*W words;
 * coeff: host or device, 2*n_terms doubles (re, im).  The data are copied;
 * the sum is not canonical until pbs_pauli_canonicalize.  Synchronizes. */
pbs_status pbs_sum_create(uint32_t n_qubits, uint64_t n_terms, const uint64_t* x, const uint64_t* z,
                          const double* coeff, void* stream, pbs_sum** out);

/* Qubit count, number of terms and whether the sum is canonical (1/0). */
pbs_status pbs_sum_info(const pbs_sum* s, uint32_t* n_qubits, uint64_t* n_terms, int32_t* canonical);

/* Copies the terms out (host or device destinations sized as in create).
 * Any destination may be NULL to skip it.  Synchronizes. */
pbs_status pbs_sum_read(const pbs_sum* s, uint64_t* x, uint64_t* z, double* coeff, void* stream);

/* Borrowed view of the sum's device arrays (Section 2.3's X, Z, C): *x and
 * *z point at n_terms*W words each (term-major, word w of term i at
 * [i*W + w], W = ceil(n_qubits / 64)), *coeff at 2*n_terms doubles (re, im,
 * letter form).  The pointers stay valid until s is destroyed or modified
 * (pbs_pauli_canonicalize); the caller must not write through them.  Any
 * output may be NULL.  An empty sum gives null array pointers.  No copy,
 * no synchronization. */
pbs_status pbs_sum_view(const pbs_sum* s, uint32_t* n_qubits, uint64_t* n_terms, const uint64_t** x,
                        const uint64_t** z, const double** coeff);

void pbs_sum_destroy(pbs_sum* s);

/* Canonical reduction in place (Section 2.3): radix sort on the (X, Z) key,
 * linear merge with correctly rounded sums, drop rule above.  Synchronizes. */
pbs_status pbs_pauli_canonicalize(pbs_sum* s, double eps_drop, void* stream);

/* Canonical product of two sums, A*B = sum_kl R(X_k^X_l, Z_k^Z_l, C_kl)
 * (Eq. pauli_operator_multiplication).  Each coefficient is the correctly
 * rounded exact value of its sum of pair products.  Requires equal qubit
 * counts and n_terms(A)*n_terms(B) < 2^30.  Synchronizes. */
pbs_status pbs_pauli_sum_mul(const pbs_sum* a, const pbs_sum* b, double eps_drop, void* stream, pbs_sum** out);

/* Jordan-Wigner qubit Hamiltonian built directly from integrals (Section 2.3,
 * Algorithm 1):
 *   H = e0 I + sum_PQ h1[P,Q] a+_P a_Q + 1/2 sum_PQRS h2[P,Q,R,S] a+_P a+_Q a_R a_S
 * (Eq. second_quantized_hamiltonian over spin-orbitals), with
 * a+_p = 1/2 (X_p - i Y_p) Z_{p-1}..Z_0 and a_p = 1/2 (X_p + i Y_p) Z_{p-1}..Z_0.
 * Each integral with |h| > eps expands into its 4 or 16 Pauli strings and
 * phase-corrected coefficients by the product rule; the contributions are
 * reduced to canonical form.
 *  n_spin_orb  1..255 (qubits).
 *  h1          device, n^2 doubles, row-major [P][Q].
 *  h2          device, n^4 doubles, row-major [P][Q][R][S] (may be NULL = 0).
 * Output: new canonical sum.  Synchronizes. */
pbs_status pbs_jw_transform(uint32_t n_spin_orb, const double* h1, const double* h2, double e0, double eps,
                            double eps_drop, void* stream, pbs_sum** out);

/* ------------------------------------------------------------------ grouping */

/* Groups a canonical sum by X-mask (Eq. topological_group): group g holds
 * X_g, its Z-masks Z_k and XZ-form coefficients C_k = c_k i^popcount(X&Z).
 * Also builds the tables of the spin-sector kernel when n_qubits is even
 * (alpha/beta split at n_qubits/2).  Requires a canonical sum with
 * n_qubits <= 64.  Synchronizes. */
pbs_status pbs_group_by_xmask(const pbs_sum* h, void* stream, pbs_grouped** out);

/* Qubit count, number of groups G and number of terms M. */
pbs_status pbs_grouped_info(const pbs_grouped* g, uint32_t* n_qubits, uint64_t* n_groups, uint64_t* n_terms);

/* Copies the CSR form out: xg [G] group masks, offsets [G+1] term offsets,
 * zk [M] Z-masks, ck [2M] XZ-form coefficients.  Host or device
 * destinations; NULL skips an array.  Synchronizes. */
pbs_status pbs_grouped_read(const pbs_grouped* g, uint64_t* xg, uint64_t* offsets, uint64_t* zk, double* ck,
                            void* stream);

void pbs_grouped_destroy(pbs_grouped* g);

/* ------------------------------------------------------------------ spaces */

/* Full space of n_qubits (1..40): D = 2^n, index = bit pattern. */
pbs_status pbs_space_full(uint32_t n_qubits, pbs_space** out);

/* Spin sector with fixed (N_alpha, N_beta) (Section 2.4; Eq. fcidim gives
 * D = C(n_orb, N_alpha) C(n_orb, N_beta)).  n_orb 1..32, D < 2^40.  Builds
 * the spin-string lists and combinatorial rank tables on the device.
 * Synchronizes. */
pbs_status pbs_space_sector(uint32_t n_orb, uint32_t n_alpha, uint32_t n_beta, void* stream, pbs_space** out);

/* Dimension D. */
pbs_status pbs_space_dim(const pbs_space* sp, uint64_t* dim);

/* Sector shape: n_orb, N_alpha, N_beta, D_alpha, D_beta (zeros and
 * PBS_ERR_ARG for a full space). */
pbs_status pbs_space_shape(const pbs_space* sp, uint32_t* n_orb, uint32_t* n_alpha, uint32_t* n_beta,
                           uint64_t* dim_alpha, uint64_t* dim_beta);

/* Index of each basis bit pattern (device arrays of n), -1 when outside the
 * space.  Asynchronous. */
pbs_status pbs_space_rank(const pbs_space* sp, uint64_t n, const uint64_t* bits, int64_t* idx, void* stream);

/* Bit pattern of each index (device arrays of n); indices outside [0, D)
 * give UINT64_MAX.  Asynchronous. */
pbs_status pbs_space_unrank(const pbs_space* sp, uint64_t n, const int64_t* idx, uint64_t* bits, void* stream);

void pbs_space_destroy(pbs_space* sp);

/* ------------------------------------------------------------------ operator-state */

/* out = P H P psi (P = projector on the space; equal to H psi for operators
 * that conserve the sector, and for any operator on the full space), by
 * target-driven summation over X-mask groups (Eq. reverse_sum; in a sector,
 * Eq. sreverse_sum): every target amplitude gathers psi[t ^ X_g] times its
 * group's phase sum, so no two threads write the same output.
 *  psi, out  device, D complex values of type dt; out must not overlap psi.
 *  The grouped operator must have the space's qubit count.
 * Asynchronous; allocates nothing. */
pbs_status pbs_apply_pauli_sum(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                               void* stream);

/* Device workspace bytes needed by pbs_expval on this space. */
pbs_status pbs_expval_workspace_bytes(const pbs_space* sp, uint64_t* bytes);

/* Energy of Eq. vqe_energy: result[0..2] = (Re <psi|H|psi>, Im <psi|H|psi>,
 * <psi|psi>), with the operator-state gather of pbs_apply_pauli_sum fused
 * into a float64 reduction (the gathered H psi is never rounded to storage
 * precision before the dot product).  When out is not NULL the same pass also
 * stores H psi there (as pbs_apply_pauli_sum would; out must not overlap psi).
 * result: device, 3 doubles; work: device workspace of at least
 * pbs_expval_workspace_bytes.  Asynchronous; allocates nothing. */
pbs_status pbs_expval(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                      double* result, void* work, uint64_t work_bytes, void* stream);

/* One share of pbs_apply_pauli_sum in a spin sector: the targets of alpha
 * rows [row_begin, row_end) only.  Target-driven summation (Eq. reverse_sum,
 * Eq. sreverse_sum) evaluates each target amplitude on its own, so the rows
 * of a sector split into independent shares that need the whole psi and no
 * reduction; a device holding one share runs this with its rows.  The same
 * kernels as the whole-sector call, so the shares concatenated are
 * bit-identical to pbs_apply_pauli_sum's output.
 *  psi  device, the whole state (D values of type dt);
 *  out  device, (row_end - row_begin) * dim_beta values: out[(a - row_begin)
 *       * dim_beta + b] is the target of alpha row a, beta column b; it must
 *       not overlap psi.
 * PBS_ERR_ARG on a full space, PBS_ERR_RANGE unless row_begin <= row_end <=
 * dim_alpha; an empty range enqueues nothing.  Asynchronous; allocates
 * nothing. */
pbs_status pbs_apply_pauli_sum_rows(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi,
                                    void* out, uint64_t row_begin, uint64_t row_end, void* stream);

/* pbs_expval over alpha rows [row_begin, row_end) of a sector: result[0..2] =
 * (Re, Im of sum over the share's targets t of conj(psi_t) (H psi)_t, and sum
 * of |psi_t|^2 over them), so that the shares' results add up to
 * pbs_expval's (up to the order of the float64 sums).  out is NULL or a
 * share as in pbs_apply_pauli_sum_rows; work: device workspace of at least
 * (row_end - row_begin) * ceil(dim_beta / 512) * 24 bytes (the whole space's
 * pbs_expval_workspace_bytes is always enough; PBS_ERR_ARG when smaller).
 * Same errors as pbs_apply_pauli_sum_rows.  Asynchronous; allocates
 * nothing. */
pbs_status pbs_expval_rows(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                           uint64_t row_begin, uint64_t row_end, double* result, void* work, uint64_t work_bytes,
                           void* stream);

/* Size of the fixed device workspace behind pbs_expval_noalloc. */
#define PBS_EXPVAL_NOALLOC_MAX_BYTES (8u * 1024u * 1024u)

/* pbs_expval without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as pbs_expval
 * (bit-identical); the per-workgroup energy partials go to a fixed array of
 * PBS_EXPVAL_NOALLOC_MAX_BYTES that the library holds on each device until
 * the process ends.  Spaces whose partials exceed it
 * (pbs_expval_workspace_bytes > PBS_EXPVAL_NOALLOC_MAX_BYTES) are refused
 * with PBS_ERR_RANGE before anything is enqueued.  Every call on one device
 * shares that device's array: calls that overlap on one device (concurrent
 * streams, or host threads racing on one stream) race on it, so serialize
 * them.  The first call on each device looks up the array's address (no
 * allocation).  Asynchronous; calls no allocating routine. */
pbs_status pbs_expval_noalloc(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, const void* psi, void* out,
                              double* result, void* stream);

/* ------------------------------------------------------------------ spin-factorized phases */

/* Spin-factorized evaluation of the phase sums (Section 2.4: Eqs.
 * svd_weights, precomp_alpha, precomp_beta, svd_sreverse_sum and dot_product;
 * Algorithm grouped_hvec; Table svd_rank_dist).  In a spin sector a group's
 * sector-form coefficients form a matrix M[mu][nu] over its alpha Z-masks and
 * beta Z-masks; with a rank-R factorization M = P Q its phase sum at
 * (t_alpha, t_beta) is sum_r A_r(t_alpha) F_r(t_beta).  This call factors
 * the operator's groups (rank-revealing Gram-Schmidt on M, relative
 * tolerance 1e-14) and precomputes F_r for every beta string of sp's
 * (n_orb, N_beta), for the X_beta = 0 group of every non-simple class and
 * for the pair and quad groups of the X_alpha = 0 class (when their ranks
 * are at most 2).  On the alpha side (Eq. precomp_alpha) it lists, for every
 * alpha string of sp's N_alpha, the simple classes (one X_beta = 0 group
 * with beta Z-masks 0) whose source lies in the sector, with their folded
 * coefficients, and the images of the classes whose pair groups have one
 * unique each (the folded coefficient per orbital pair and the class's
 * X_beta = 0 factors).  The tables are attached to h (replacing earlier ones);
 * afterwards pbs_apply_pauli_sum, pbs_expval and batch jobs on sectors with
 * the same (n_orb, N_beta), respectively (n_orb, N_alpha) for the alpha
 * lists, use them (results equal the unfactored evaluation up to rounding).
 * Needs real sector-form coefficients (PBS_ERR_UNSUPPORTED otherwise) and a
 * sector space with n_orb = n_qubits / 2.  Allocates the tables (device
 * memory owned by h) and synchronizes the stream; must not run while h is
 * in use by another call. */
pbs_status pbs_grouped_factor(pbs_grouped* h, const pbs_space* sp, void* stream);

/* Chooses which of h's factor tables later single applies and energies use:
 * mode bit 0 the rows of the X_beta = 0 groups, bit 1 the move tables of the
 * X_alpha = 0 class, bit 2 the alpha lists of the simple classes (7, all, is
 * the default; 0 turns the factored evaluation off).  Batches use the same mode unless the
 * PBS_BATCH_NO_FACTORED schedule bit is set.  Must not run while h is in use. */
pbs_status pbs_grouped_set_factored(pbs_grouped* h, int32_t mode);

/* info[0..10] (host): tables present (0/1), X_beta = 0 groups factored,
 * their largest rank, X_alpha = 0 pair groups factored, their rank, its quad
 * groups factored, their rank, the N_beta the tables are for, alpha lists
 * present (0/1), the N_alpha they are for, alpha images present (0/1). */
pbs_status pbs_grouped_factor_info(const pbs_grouped* h, uint32_t* info);

/* ------------------------------------------------------------------ batched apply */

/* Prepares one launch that applies n operators to n states in spin sectors:
 * job i computes out[i] = P h[i] P psi[i] on sp[i] exactly as
 * pbs_apply_pauli_sum does (target-driven summation, Eq. sreverse_sum), with
 * every job's workgroups in a single grid (largest jobs first).  Sectors may
 * differ in size and shape, and each job has its own operator.
 *  h, sp, psi, out  host arrays of n handles / device pointers; all states
 *                   have storage type dt; out[i] must not overlap psi[i] or
 *                   any other job's output.  The pointers are recorded: the
 *                   batch always runs on these buffers.
 * Allocates the job table and a partial-sum buffer once.  Synchronizes. */
pbs_status pbs_batch_create(uint32_t n, const pbs_grouped* const* h, const pbs_space* const* sp, pbs_dtype dt,
                            const void* const* psi, void* const* out, pbs_batch** batch);

/* Runs a prepared batch on the stream.  With energies == NULL only the
 * products are written; otherwise the same single pass also writes, for each
 * job i, energies[3i..3i+2] = (Re <psi|H|psi>, Im <psi|H|psi>, <psi|psi>)
 * accumulated in float64 (device array of 3n doubles).  Asynchronous;
 * allocates nothing and may be captured in a HIP graph.  Two runs of one
 * batch must not overlap in time (they share the partial-sum buffer). */
pbs_status pbs_batch_run(const pbs_batch* b, double* energies, void* stream);

/* Schedule of a batched launch: bits of `config` (0 = the default schedule).
 * Every schedule computes the same products and energies up to the order of
 * floating-point additions within a target; the workgroup order alone
 * changes no output bit. */
#define PBS_BATCH_GIVEN_ORDER 1u       /* jobs in the caller's order (default: largest first) */
#define PBS_BATCH_NO_ROW_STAGING 2u    /* gather source rows from HBM/L2 instead of staging them in LDS */
#define PBS_BATCH_NO_DOUBLE_MOVES 4u   /* scan double-flip groups instead of enumerating double moves */
#define PBS_BATCH_NO_SINGLE_MOVES 8u   /* scan pair groups instead of enumerating single moves */
#define PBS_BATCH_NO_FACTORED 64u      /* ignore the operators' factor tables (pbs_grouped_factor) */
#define PBS_BATCH_PERSISTENT 128u      /* persistent launch: as many workgroups as are resident at once,
                                          each walking the (largest-first) work list with a fixed stride */
/* workgroup -> (alpha row, beta chunk) order of every job (bits 4-5); the
 * default is the single launch's: rows fastest when rows are staged in LDS,
 * else a row's chunks kept together on one XCD (shared L2) */
#define PBS_BATCH_ORDER_MASK 48u
#define PBS_BATCH_ORDER_PLAIN 16u      /* row-major: a row's chunks consecutive */
#define PBS_BATCH_ORDER_ROW_FAST 32u   /* rows fastest */
#define PBS_BATCH_ORDER_XCD_ROWS 48u   /* a row's chunks on one XCD */

/* Rebuilds the batch's job table for schedule `config` (0..255).  Synchronizes. */
pbs_status pbs_batch_set_config(pbs_batch* b, uint32_t config);

/* Autotuner: times schedules (a warm-up run, then `reps` runs, 1..100, with
 * HIP events on the stream; schedules that build the same job table are
 * timed once), greedily: the four workgroup orders with the default flags,
 * then the 64 flag combinations with the best order.  Keeps the fastest and
 * returns it in *config and its time per run in *ms (either may be NULL).
 * Runs the batch, so the output buffers are overwritten.  Call it before
 * capturing pbs_batch_run in a graph: it rebuilds the job table.
 * Synchronizes. */
pbs_status pbs_batch_tune(pbs_batch* b, uint32_t reps, void* stream, uint32_t* config, double* ms);

/* Schedule in use, its tuned time per run (-1 when not chosen by the tuner)
 * and the number of workgroups of one launch.  Any output may be NULL. */
pbs_status pbs_batch_info(const pbs_batch* b, uint32_t* config, double* tuned_ms, uint32_t* workgroups);

void pbs_batch_destroy(pbs_batch* b);

/* ------------------------------------------------------------------ propagation */

/* Device workspace bytes for pbs_krylov_step with m Krylov vectors (1..16):
 * m + 1 state vectors of type dt plus reduction scratch. */
pbs_status pbs_krylov_workspace_bytes(const pbs_space* sp, pbs_dtype dt, uint32_t m, uint64_t* bytes);

/* One real-time step psi <- exp(-i H dt_step) psi (Section 2.1,
 * Eq. real_time_evolution) by short-iterative Lanczos: up to m Krylov vectors
 * built with pbs_apply_pauli_sum's kernels, the three-term recurrence and
 * one full classical Gram-Schmidt re-orthogonalisation per vector with
 * float64 inner products, exp(-i T dt) e_1 of the tridiagonal
 * T from its eigen-decomposition, psi rebuilt as |psi| V exp(-i T dt) e_1.
 * The basis stops early when the new vector's norm falls below 1e-14 times
 * the largest entry of T (the Krylov space is then invariant and the step is
 * exact).  H must be Hermitian.
 *  psi    device, D complex values of type dt, updated in place.
 *  work   device workspace of at least pbs_krylov_workspace_bytes; must not
 *         overlap psi.
 *  info   host, 4 doubles: |psi| before the step, <H> of the normalised input
 *         state, number of Krylov vectors used, norm of the last residual.
 * Synchronizes the stream (the tridiagonal matrix is read back). */
pbs_status pbs_krylov_step(const pbs_grouped* h, const pbs_space* sp, pbs_dtype dt, void* psi, double dt_step,
                           uint32_t m, void* work, uint64_t work_bytes, double* info, void* stream);

/* ------------------------------------------------------------------ variational layer */

/* Ansatz psi(theta) = R_{n-1} ... R_0 |ref>, R_k = exp(i theta_k P_k) =
 * cos(theta_k) + i sin(theta_k) P_k, over the full 2^(2 n_orb) space, with
 * its energy <psi|H|psi> (Section 2.1, Eq. vqe_energy).  H must conserve
 * N_alpha and N_beta (a JW Hamiltonian of spin-orbital integrals): the
 * product H|psi> runs through the batched sector kernel over all
 * (N_alpha, N_beta) blocks of the full space.  This is checked on the
 * grouped terms when the handle is created: an operator with a sector-changing
 * part (a pairing term, a lone X_p X_q) is refused with PBS_ERR_UNSUPPORTED
 * rather than having that part dropped.
 *  h      grouped operator on 2 n_orb qubits (1 <= n_orb <= 14), with sector
 *         tables; it must outlive the handle.
 *  n_rot  number of rotations, 0..4096 (PBS_ERR_RANGE beyond).
 *  x, z   host, n_rot words: the Hermitian letter-form strings P_k (phase 0).
 *  ref    basis index of the reference state (bit k = qubit k).
 *  dt     storage of the state vectors; energies, overlaps and gradients are
 *         float64.
 * Allocates four full-space vectors and the sector tables; synchronizes the
 * stream. */
pbs_status pbs_vqe_create(const pbs_grouped* h, uint32_t n_orb, uint32_t n_rot, const uint64_t* x, const uint64_t* z,
                          uint64_t ref, pbs_dtype dt, void* stream, pbs_vqe** out);

/* energy = <psi(theta)|H|psi(theta)>; when grad is not NULL, also
 * grad[k] = dE/dtheta_k = -2 Im <lambda_k|P_k|psi_k> by the adjoint method
 * (psi_k after rotation k, lambda_k = R_{k+1}^dag ... R_{n-1}^dag H psi).
 * theta, energy, grad: host.  Synchronizes the stream.  Calls on one handle
 * must not overlap. */
pbs_status pbs_vqe_energy_grad(pbs_vqe* v, const double* theta, double* energy, double* grad, void* stream);

/* Writes psi(theta) of the last pbs_vqe_energy_grad call (2^(2 n_orb)
 * values of the handle's dtype, full-space order) to the device buffer
 * psi_out.  PBS_ERR_ARG before the first evaluation. */
pbs_status pbs_vqe_state(const pbs_vqe* v, void* psi_out, void* stream);

/* Minimises the energy over theta (host, n_rot doubles, in/out: start point
 * in, minimiser out) with pbs_lbfgs_minimize, each evaluation being one
 * pbs_vqe_energy_grad call on the stream; the decrease test tolerates
 * 1e-13 (complex128) or 1e-6 (complex64) relative noise in E.  Outputs as in pbs_lbfgs_minimize
 * (energy = final E).  Synchronizes. */
pbs_status pbs_vqe_minimize(pbs_vqe* v, double* theta, uint32_t max_iter, double g_tol, double f_tol, void* stream,
                            double* energy, uint32_t* iters, uint32_t* evals, int32_t* reason);

/* Runs pbs_batch_tune on the handle's batched launch over the sector blocks
 * (after at least one evaluation) and keeps the fastest schedule; *config and
 * *ms as there.  pbs_vqe_set_config applies a known schedule (for example
 * one tuned at another geometry of the same shape).  Both synchronize. */
pbs_status pbs_vqe_tune(pbs_vqe* v, uint32_t reps, void* stream, uint32_t* config, double* ms);
pbs_status pbs_vqe_set_config(pbs_vqe* v, uint32_t config);

/* Most consecutive rotations applied in one pass over the state (forward
 * sweep) and undone in one pass over state and adjoint (gradient sweep), each
 * 1, 2 or 3; rotations are fused when their X masks are linearly
 * independent.  The results do not depend on it beyond rounding. */
pbs_status pbs_vqe_set_groups(pbs_vqe* v, uint32_t forward, uint32_t adjoint);

/* Number of (N_alpha, N_beta) blocks of the handle, and how many of them are
 * stored and applied as sector (N_beta, N_alpha): blocks with fewer beta than
 * alpha strings and fewer than 512 beta strings, when the operator maps onto
 * itself term by term under exchanging the two qubit halves (spin-free
 * integrals).  Either output may be NULL. */
pbs_status pbs_vqe_info(const pbs_vqe* v, uint32_t* n_blocks, uint32_t* n_transposed);

void pbs_vqe_destroy(pbs_vqe* v);

/* ------------------------------------------------------------------ optimizer */

/* Objective for pbs_lbfgs_minimize: writes f(x) and its gradient g (n
 * doubles, host) and returns 0, or nonzero to abort the minimisation. */
typedef int32_t (*pbs_objective)(void* user, uint32_t n, const double* x, double* f, double* g);

/* Limited-memory BFGS (host code) with a strong-Wolfe line search
 * (c1 = 1e-4, c2 = 0.9), the optimiser of the paper's VQE runs (Section 3.2);
 * the decrease test tolerates 1e-13 max(|f|, 1) of rounding noise in f.
 * x: host, n doubles, start point in, final point out.  history: curvature
 * pairs kept (1..64).  Stops with *reason = 0 when max |g_i| <= g_tol, 1 when
 * (f_tol > 0) an accepted step lowers f by at most
 * f_tol * max(|f_old|, |f_new|, 1), 2 at
 * max_iter iterations, 3 when the line search finds no acceptable step.
 * f_out, iters, evals (objective calls), reason may be NULL.  An objective
 * failure returns PBS_ERR_ARG. */
pbs_status pbs_lbfgs_minimize(uint32_t n, double* x, pbs_objective fn, void* user, uint32_t max_iter,
                              uint32_t history, double g_tol, double f_tol, double* f_out, uint32_t* iters,
                              uint32_t* evals, int32_t* reason);

/* ------------------------------------------------------------------ warm-start network */

/* A 1 -> H -> H -> O perceptron that maps a geometry coordinate R of a
 * potential-energy scan to ansatz parameters theta(R), trained on converged
 * parameters of earlier geometries (an extension beyond the paper, which
 * optimises each geometry from scratch, Section 3.2):
 *   h1 = tanh(W1 R + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3,
 * loss = mean over rows and outputs of (y - t)^2, full-batch Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * Every product rounds its operands to bfloat16 (nearest-even) and
 * accumulates in float32 on the matrix cores; parameters, Adam moments,
 * activations and bias gradients are float32.
 * Parameters are one float32 array packed as
 *   [W1 (H), b1 (H), W2 (H*H, row j = unit j), b2 (H), W3 (O*H), b3 (O)];
 * gradients use the same layout. */

/* Number of packed parameters for hidden width H and output width O. */
pbs_status pbs_mlp_param_count(uint32_t hidden, uint32_t n_out, uint64_t* count);

/* hidden: multiple of 32 in 32..1024; n_out 1..1024; max_batch 1..4096 rows.
 * params: host or device, packed initial parameters (copied).  Adam state
 * starts at zero.  Allocates every buffer the other calls use.  Synchronizes. */
pbs_status pbs_mlp_create(uint32_t hidden, uint32_t n_out, uint32_t max_batch, const float* params, void* stream,
                          pbs_mlp** out);

/* Replaces the parameters (host or device source) and resets Adam.  Synchronizes. */
pbs_status pbs_mlp_set_params(pbs_mlp* m, const float* params, void* stream);

/* Copies the parameters to a host or device array.  Synchronizes. */
pbs_status pbs_mlp_get_params(const pbs_mlp* m, float* params, void* stream);

/* Inference: y[n][O] (device, row-major) for inputs x[n] (device), 1 <= n <= max_batch.
 * Asynchronous.  Calls on one handle must not overlap (shared activations). */
pbs_status pbs_mlp_forward(pbs_mlp* m, uint32_t n, const float* x, float* y, void* stream);

/* Loss and gradient without an update: targets t[n][O] (device), loss (device
 * float, may be NULL), grad (device, packed layout).  Asynchronous. */
pbs_status pbs_mlp_loss_grad(pbs_mlp* m, uint32_t n, const float* x, const float* t, float* loss, float* grad,
                             void* stream);

/* n_steps full-batch Adam steps with learning rate lr on (x, t), continuing
 * the handle's step count; losses (device, n_steps floats, may be NULL)
 * receives the loss before each step of this call.  Asynchronous: a one-thread
 * kernel marks the start of the call, then nine kernel launches per step on
 * the caller's stream.  The step count and the call's first step are kept on
 * the device and loss slots are bounded by n_steps, so a call allocates
 * nothing, copies nothing and may be captured in a HIP graph by the caller:
 * each replay, and each direct call after replays, continues the count and
 * writes losses[0 .. n_steps-1] of its own buffer. */
pbs_status pbs_mlp_train(pbs_mlp* m, uint32_t n, const float* x, const float* t, uint32_t n_steps, float lr,
                         float* losses, void* stream);

void pbs_mlp_destroy(pbs_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* PBS_H_ */
