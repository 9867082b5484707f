/*
 * zx.h -- C ABI of libzx: bit-packed GF(2) work on graph-like ZX diagrams
 * for AMD MI355X (gfx950).
 *
 * Paper: "Tsim: Fast Universal Simulator for Quantum Error Correction"
 * (arXiv 2604.01059).  Operations and the passages that define them:
 *   local complementation  appendix "Rewrite rules", equation local_comp
 *   pivoting               appendix "Rewrite rules", equation pivoting
 *   simplification         stops when no interior pi/2 spider and no pair of
 *                          adjacent interior pi spiders remains (appendix
 *                          "Stabilizer decompositions", first paragraph);
 *                          cost cubic in the spider count (section
 *                          "Complexity", paragraph "Compilation")
 *   GF(2) elimination      Gaussian elimination over F2 to a linearly
 *                          independent basis (section on the repetition-code
 *                          example, sentence after equation detector_sampling)
 *   Pauli encoding         two bits per qubit, (x,z) = (1,0) X, (1,1) Y,
 *                          (0,1) Z (appendix "Pauli channels", equation
 *                          channel_pauli1 and the sentence after it)
 *
 * Conventions for every call
 *   - Device memory is owned by the caller.  The library allocates no device
 *     memory; scratch space comes from caller workspaces whose size the
 *     matching *_workspace_bytes() call returns.  Host pointers are read
 *     during the call only.
 *   - Calls are asynchronous on the given stream unless documented as
 *     synchronising.  The stream may be NULL (the null stream).
 *   - Return value: ZX_OK or a negative zx_status.  Argument errors are
 *     detected on the host and returned immediately; errors found by a
 *     kernel (a rule whose precondition does not hold, a capacity overflow,
 *     a spin-wait time-out) are recorded in a sticky status word that the
 *     *_status() calls read.  zx_last_error() describes the most recent host
 *     error of the calling thread.  No C++ exception crosses this boundary.
 *   - Bit matrices are row-major arrays of uint64_t words: bit c of row r is
 *     bit (c % 64) of word r * ld + c / 64.
 */
#ifndef ZX_H
#define ZX_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t zx_status;
#define ZX_OK 0
#define ZX_EINVAL (-1)     /* bad argument (host-detected) */
#define ZX_ENOMATCH (-2)   /* rule precondition false (device-detected) */
#define ZX_ECAPACITY (-3)  /* size beyond what a kernel or workspace supports */
#define ZX_EDEVICE (-4)    /* HIP runtime error or device spin-wait time-out */
#define ZX_EBUSY (-5)      /* admission refused: budget exhausted */

/* flags */
#define ZX_GRAPH_ONLY 0x1u   /* rewrites: only the edge toggles, keep vertices/phases */
#define ZX_SYNC 0x100u       /* synchronise the stream before returning */

/* Version of the ABI (major * 100 + minor). */
int32_t zx_version(void);
/* Thread-local description of the last host-side error ("" if none). */
const char* zx_last_error(void);
/* Number of kernels and the device name the library will launch on. */
zx_status zx_device_info(char* name, int32_t name_len, int32_t* n_cu);

/* ======================================================================
 * Graph-like diagrams
 *
 * A diagram lives in one caller-allocated device arena of zx_graph_bytes()
 * bytes.  It holds:
 *   - the SOURCE diagram given to zx_graph_create (read-only afterwards);
 *   - the CURRENT diagram: adjacency n x W (W = ceil(n/64)), phases k
 *     (int8, units of pi/4, 0..7), alive mask, scalar
 *     omega^phase8 * sqrt(2)^pow_sqrt2 (omega = e^{i pi/4}) multiplying the
 *     diagram's linear map;
 *   - the rewrite trace and the extracted output frontier.
 * Spiders are Z spiders joined by Hadamard edges.  Boundary wires are kept
 * outside the adjacency: input i attaches to spider in_spider[i], output j to
 * out_spider[j]; a spider carrying a boundary wire is never rewritten.
 * ==================================================================== */
typedef struct zx_graph zx_graph;

typedef struct {
  int64_t pow_sqrt2;   /* scalar: power of sqrt(2) */
  int32_t phase8;      /* scalar: power of omega, 0..7 */
  int32_t status;      /* sticky device status of this graph (zx_status) */
  int32_t n;           /* spiders (rows of the adjacency) */
  int32_t n_alive;     /* spiders still present */
  int64_t n_edges;     /* Hadamard edges among present spiders */
  int32_t n_trace;     /* rewrites recorded by the last zx_simplify */
  int32_t rounds;      /* rewrite rounds of the last zx_simplify */
  int64_t fill_in;     /* edges toggled on by rewrites */
  int32_t rank;        /* rank of the output frontier (-1 if not extracted) */
  int32_t policy;      /* schedule of the CURRENT diagram (ZX_POLICY_*) */
  int64_t rowops;      /* row additions of the frontier elimination */
} zx_graph_info;

/* Arena size for a diagram of n spiders with n_in inputs and n_out outputs. */
size_t zx_graph_bytes(int32_t n, int32_t n_in, int32_t n_out);

/* Create a diagram in dev_arena (device memory, >= zx_graph_bytes, 256-byte
 * aligned).  adj_host: n x ceil(n/64) words, symmetric, zero diagonal, bits
 * >= n zero.  phase_host: n values in 0..7.  in_spider/out_spider: distinct
 * spider ids per boundary wire.  bnd_is_hadamard: n_in + n_out flags (NULL =
 * all plain wires).  The host handle *g is freed by zx_graph_destroy; the
 * arena stays the caller's.  Copies host->device on stream s. */
zx_status zx_graph_create(zx_graph** g, void* dev_arena, size_t arena_bytes, int32_t n,
                          const uint64_t* adj_host, const int8_t* phase_host,
                          const int32_t* in_spider, int32_t n_in,
                          const int32_t* out_spider, int32_t n_out,
                          const uint8_t* bnd_is_hadamard, hipStream_t s);
/* Parameterized Pauli spiders (Pauli boxes).  The paper models Pauli noise
 * as spiders whose phase carries a binary parameter times pi (section on the
 * ZX representation; the rewrite rules of appendix "Rewrite rules" are
 * stated for phases pi/2 + b pi and a pi with binary a, b).  Here spider v's
 * phase is k_v pi/4 + (p_v . f) pi, p_v its parameter row: n_params bits in
 * pw = ceil(n_params/64) words, param_rows n x pw words (host), bits at or
 * beyond n_params zero.  n_params <= 4096.  Rewrites never look at the
 * parameters to decide (the schedule is that of the constant phases); they
 * update the rows (local complementation at u XORs p_u into every neighbour;
 * a pivot u-v XORs p_v into N(u) only, p_u into N(v) only, both into common
 * neighbours) and, when a rewrite's scalar depends on the parameters, record
 * a phase-pair term (k_alpha, k_beta, u, v): the factor
 * h(k_alpha pi/4, k_beta pi/4; u.f, v.f) of the parameterized evaluation
 * appendix (equation phase_pair).  For every f the CURRENT diagram then
 * satisfies  D_source(f) = omega^phase8 sqrt(2)^pow_sqrt2 prod_terms h * D(f).
 * Local complementation with p_u != 0 gives (4, 2, p_u, 0) if k_u = 2,
 * (0, 2, p_u, 0) if k_u = 6; a pivot with p_u or p_v != 0 gives
 * (k_u, k_v, p_u, p_v).  zx_graph_bytes_ex / zx_graph_create_ex take the
 * parameters; with n_params = 0 they equal zx_graph_bytes / zx_graph_create.
 * Serving requests carry no parameters. */
size_t zx_graph_bytes_ex(int32_t n, int32_t n_in, int32_t n_out, int32_t n_params);
zx_status zx_graph_create_ex(zx_graph** g, void* dev_arena, size_t arena_bytes, int32_t n,
                             const uint64_t* adj_host, const int8_t* phase_host,
                             const int32_t* in_spider, int32_t n_in,
                             const int32_t* out_spider, int32_t n_out,
                             const uint8_t* bnd_is_hadamard, int32_t n_params,
                             const uint64_t* param_rows, hipStream_t s);
/* CURRENT parameter rows (n x pw words) and the terms recorded since the
 * SOURCE diagram (count to *n_terms; the first min(count, cap) to k_ab
 * (2 int32 each: k_alpha, k_beta), u and v (pw words each)), in the order of
 * the rewrites that made them.  Any output may be NULL.  Synchronises s. */
zx_status zx_graph_read_params(const zx_graph* g, uint64_t* rows, int32_t* n_terms, int32_t* k_ab,
                               uint64_t* u, uint64_t* v, int32_t cap, hipStream_t s);
/* Attach a handle to an arena already initialised by zx_graph_create. */
zx_status zx_graph_attach(zx_graph** g, void* dev_arena, size_t arena_bytes);
void zx_graph_destroy(zx_graph* g);   /* host handle only */
void* zx_graph_arena(const zx_graph* g);

/* Copy the CURRENT diagram to host buffers (any may be NULL).  Synchronises s.
 * adj: n x W words; phase: n bytes; alive: W words. */
zx_status zx_graph_read(const zx_graph* g, uint64_t* adj, int8_t* phase, uint64_t* alive,
                        zx_graph_info* info, hipStream_t s);
/* Trace of the last zx_simplify: n_trace entries {round, rule, u, v},
 * rule 0 = local complementation (v = -1), 1 = pivot.  Synchronises s. */
zx_status zx_graph_read_trace(const zx_graph* g, int32_t* trace, int32_t cap,
                              int32_t* n_trace, hipStream_t s);
/* Output frontier after zx_simplify with extraction: n_out x W words in
 * reduced row echelon form and n_out pivot columns (-1 padded).  Synchronises. */
zx_status zx_graph_read_frontier(const zx_graph* g, uint64_t* rows, int32_t* pivots,
                                 hipStream_t s);
/* Sticky device status of the graph (synchronises s). */
zx_status zx_graph_status(const zx_graph* g, hipStream_t s);
/* Make the CURRENT diagram equal to the SOURCE diagram again (async). */
zx_status zx_graph_reset(zx_graph* g, hipStream_t s);

/* Local complementation at spider u on the CURRENT diagram (rule above).
 * Precondition (checked on the device): u present, no boundary wire, phase
 * pi/2 or 3pi/2.  If it fails nothing changes and the graph's status becomes
 * ZX_ENOMATCH.  flags & ZX_GRAPH_ONLY: complement the edges among N(u) only
 * (u must be present; phases, scalar and u are kept). */
zx_status zx_local_comp(zx_graph* g, int32_t u, uint32_t flags, hipStream_t s);
/* Pivot on the edge u-v of the CURRENT diagram (rule above).  Precondition
 * (device): u ~ v, both present without boundary wire, phases 0 or pi.
 * ZX_GRAPH_ONLY: complete tripartite toggle between N(u) only, N(v) only and
 * common neighbours; u and v are kept. */
zx_status zx_pivot(zx_graph* g, int32_t u, int32_t v, uint32_t flags, hipStream_t s);

/* ======================================================================
 * Simplification to the rules' fixed point
 *
 * zx_simplify starts from each graph's SOURCE diagram (so it can be re-run),
 * writes the result into the CURRENT diagram, the trace, and with extract=1
 * the reduced output frontier.  Schedule (deterministic, bit-exact with the
 * CPU reference): local-complementation rounds, then pivot rounds.  An LC
 * round takes, in ascending spider id, every candidate not adjacent to one
 * already taken; a pivot round takes, in lexicographic order, every
 * candidate edge whose ends are distinct from and not adjacent to the ends
 * already taken.  All rewrites of a round are applied together.
 * ==================================================================== */
#define ZX_POLICY_GREEDY 0
/* Learned priority (policy ZX_POLICY_LEARNED): the phases stay those of the
 * canonical schedule.  A local-complementation round lists its candidate
 * spiders (ascending), scores each with the network in opts.mlp on the
 * features described at zx_rollout, and takes them in descending score order
 * (ties: list order) unless adjacent to one already taken.  A pivot round
 * lists the candidate edges u < v between Pauli spiders (lexicographic, at
 * most max(64, n) rounded up to a power of two), scores them the same way,
 * takes them in that order unless an end is taken or adjacent to a taken
 * end, then completes the round with the canonical lexicographic pass over
 * the edges left (so the round is maximal).  Results are exact ZX rewrites
 * whatever the scores; only the schedule differs. */
#define ZX_POLICY_LEARNED 1
#define ZX_RESUME 0x2u   /* continue from the CURRENT diagram, trace and round count */
/* Greedy fallback (with ZX_POLICY_LEARNED): per diagram, the greedy schedule
 * also runs (its result is not kept), and the CURRENT diagram ends as the
 * learned result when its gate2q -- Hadamard edges left plus, with extract,
 * the row additions of the output frontier -- is not above the greedy one,
 * else as the greedy result (the greedy schedule runs again to write it,
 * trace included).  A diagram beyond the learned policy's LDS budget, or
 * whose learned run fails on the device, gets the greedy result.
 * zx_graph_info.policy tells which schedule the arena holds.  Not combined
 * with max_rounds or ZX_RESUME (ZX_EINVAL). */
#define ZX_FALLBACK 0x4u

typedef struct zx_mlp zx_mlp;

typedef struct {
  int32_t policy;       /* ZX_POLICY_GREEDY or ZX_POLICY_LEARNED */
  int32_t extract;      /* 1 = also reduce the output frontier */
  int32_t tune_id;      /* kernel variant, -1 = autotuned / default */
  uint32_t flags;       /* ZX_SYNC, ZX_RESUME */
  int32_t max_rounds;   /* stop after this many rounds in total, 0 = fixed point */
  int32_t pad;
  const zx_mlp* mlp;    /* ZX_POLICY_LEARNED: the scoring network */
} zx_simplify_opts;

/* Number of kernel variants and a short description of variant id
 * ("bs<threads>-lds<KiB>k").  The one-wavefront variant (bs64) runs the
 * greedy schedule only: with ZX_POLICY_LEARNED it is refused as too small
 * (ZX_ECAPACITY).  Without a tune_id, a batch of up to 256 diagrams of at
 * most 64 spiders takes it; such diagrams without parameters run their
 * whole greedy simplification and frontier in one wavefront's registers. */
int32_t zx_simplify_variants(void);
const char* zx_simplify_variant_name(int32_t id);

/* Workspace for a batch of n_graphs diagrams. */
size_t zx_simplify_workspace_bytes(int32_t n_graphs);

/* One persistent launch over all graphs (uploads the batch descriptor into
 * ws first, synchronously).  Larger diagrams are scheduled first. */
zx_status zx_simplify(zx_graph* const* graphs, int32_t n_graphs, const zx_simplify_opts* o,
                      void* ws, size_t ws_bytes, hipStream_t s);

/* Batch plans: prepare once (uploads the descriptor table into ws,
 * synchronous), then launch any number of times with zx_batch_simplify,
 * which only enqueues kernels and may be captured into a HIP graph. */
typedef struct zx_batch zx_batch;
zx_status zx_batch_prepare(zx_batch** b, zx_graph* const* graphs, int32_t n_graphs,
                           void* ws, size_t ws_bytes, hipStream_t s);
zx_status zx_batch_simplify(zx_batch* b, const zx_simplify_opts* o, hipStream_t s);
/* Worst sticky status over the batch's graphs (synchronises). */
zx_status zx_batch_status(zx_batch* b, hipStream_t s);
/* Time every variant on this batch (reps launches each, after one warm-up)
 * and return the fastest id; results are cached per (device, size class). */
zx_status zx_batch_autotune(zx_batch* b, int32_t extract, int32_t reps, int32_t* best_id,
                            float* best_ms, hipStream_t s);
void zx_batch_destroy(zx_batch* b);

/* ======================================================================
 * GF(2) reduced row echelon form (Gauss-Jordan elimination over F2, as the
 * paper uses to keep a linearly independent basis of a binary matrix:
 * detectors/observables section, around equation detector_sampling)
 *
 * R = RREF(A) for an m x n_cols bit matrix (ld words per row; bits >= n_cols
 * are ignored and written as zero).  A and R may be the same buffer (in
 * place); otherwise they must not overlap.  rank_dev: one device int32.
 * pivot_cols_dev: m device int32, pivot column of output row i, -1 for rows
 * beyond the rank.
 * T (optional, NULL = none): m x ld_t words (ld_t >= ceil(m/64)), written
 * with an invertible transform such that T * A = R over F2: its first rank
 * rows give the reduced pivot rows as combinations of A's rows, the others
 * (rows of A that are no pivot, ascending) span the left null space.  T is
 * unique when A has full row rank; it must not overlap A or R.
 * One cooperative persistent launch: every word column (of A, and of T when
 * requested) lives in one workgroup's LDS, so m * 8 bytes per column must fit
 * (m <= 16384) and the grid must be co-resident; otherwise ZX_ECAPACITY.
 * Device buffers are the caller's; the call only reads A and writes R, T,
 * rank, pivots and the workspace.  Asynchronous on s.
 * ==================================================================== */
size_t zx_gf2_workspace_bytes(int32_t m, int32_t n_cols);
zx_status zx_gf2_eliminate(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols,
                           int64_t ld_words, int32_t* rank_dev, int32_t* pivot_cols_dev,
                           uint64_t* T, int64_t ld_t, void* ws, size_t ws_bytes, hipStream_t s);
/* Allocation-free elimination, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as
 * zx_gf2_eliminate, without ws: the workspace is a static device array of
 * the library, sized for m <= 16384 (658,176 bytes on every GPU the library
 * runs on, held until the process ends; larger m returns ZX_ECAPACITY).  The
 * call itself allocates nothing; its first call on a device looks up that
 * device's copy of the array.  Every call on one GPU shares the array, which
 * keeps the last call's contents: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.  No
 * per-strip profile.  *rank_dev is -1 after the stream completes if the
 * kernel detected a failure (spin-wait time-out). */
zx_status zx_gf2_eliminate_noalloc(const uint64_t* A, uint64_t* R, int32_t m, int32_t n_cols,
                                   int64_t ld_words, int32_t* rank_dev, int32_t* pivot_cols_dev,
                                   uint64_t* T, int64_t ld_t, hipStream_t s);
/* Sticky status of the last elimination that used this workspace (syncs). */
zx_status zx_gf2_status(const void* ws, hipStream_t s);
/* Per-strip timestamps (100 MHz real-time counter) of the last elimination in
 * this workspace, recorded only when the environment variable
 * ZX_RREF_PROFILE=1 was set when the library first launched the kernel.
 * ticks: n x 8 int64 (n = min(max_strips, strips recorded)); per strip t:
 * [0] owner starts, [1] candidates ready, [6] reduction done, [2] pass
 * published, [3] owner applied it, [4] next owner saw the strip's last pass,
 * [5] next owner applied it.  Unrecorded slots are 0.  Synchronises s. */
zx_status zx_gf2_profile_read(const void* ws, int32_t m, int64_t* ticks, int32_t max_strips,
                              hipStream_t s);

/* ======================================================================
 * Symplectic commutation table of Pauli strings
 *
 * X, Z: n_paulis x ld_q words (device); qubit b of string i is bit b of the
 * X and Z rows (bits at or beyond n_qubits are ignored).  C: n_paulis x ld_c
 * words (device, ld_c >= ceil(n/64)), C[i][j] = parity of
 * sum_b x_i[b] z_j[b] + z_i[b] x_j[b], i.e. 1 when strings i and j
 * anticommute.  Bits beyond n_paulis in a row are zero; words at or beyond
 * ceil(n/64) are not written.
 * Variants: ZX_PAULI_FORCE_VALU, bitwise AND/XOR on the vector units;
 * ZX_PAULI_FORCE_MFMA, the same product on the matrix cores (bits as FP4
 * values, exact fp32 counts, see zx_gf2_matmul).  ZX_PAULI_AUTO takes the
 * matrix cores from 1024 strings up.  Both give identical bits.
 * ==================================================================== */
#define ZX_PAULI_AUTO 0u
#define ZX_PAULI_FORCE_VALU 0x1u
#define ZX_PAULI_FORCE_MFMA 0x2u
zx_status zx_pauli_commute(const uint64_t* X, const uint64_t* Z, int64_t n_paulis,
                           int32_t n_qubits, int64_t ld_q, uint64_t* C, int64_t ld_c,
                           uint32_t flags, hipStream_t s);

/* ======================================================================
 * Parameterized evaluation: batched parities and the phase-pair product
 *
 * After reduction, a diagram with parameterized Pauli spiders evaluates to
 * c * prod_k h(alpha_k, beta_k; a_k, b_k), where a_k and b_k are parities of
 * the binary parameters f (appendix "Parameterized evaluation of Clifford
 * ZX diagrams", equations parities, phase_pair and scalar_product).
 * ==================================================================== */
/* C[i][j] = (sum_{b < k_bits} A[i][b] B[j][b]) mod 2: row i of A selects
 * parameters (u_i), row j of B is one parameter setting (f_j), so C holds
 * a_i for every setting j (equation parities batched over settings).
 * A: m x lda words, B: n x ldb words, C: m x ldc words (ldc >= ceil(n/64);
 * words at or beyond ceil(n/64) are not written), all device memory.  Bits at
 * or beyond k_bits are ignored; bits beyond n in a row of C are zero.  Runs
 * on the matrix cores: bits enter as FP4 values 0 and 1 and every sum is an
 * exact fp32 count.  flags: ZX_SYNC only.  Asynchronous on s. */
zx_status zx_gf2_matmul(const uint64_t* A, int64_t m, int64_t lda, const uint64_t* B, int64_t n,
                        int64_t ldb, int32_t k_bits, uint64_t* C, int64_t ldc, uint32_t flags,
                        hipStream_t s);
/* Minimal parameter basis (section on the repetition-code example: after
 * equation detector_sampling, a minimal set of f is chosen by Gaussian
 * elimination over F2 of the parameter dependencies, keeping a linearly
 * independent basis).  D: m x ld words, one dependency vector per row
 * (n_cols bits: the parameter rows left after reduction and the terms'
 * u and v).  R (m x ld, must not overlap D) receives RREF(D); its first
 * *rank_dev rows are the basis T, f = T e.  coeff (m x ldc words, ldc >=
 * ceil(min(m, n_cols)/64)) receives each vector's coordinates in that basis:
 * bit j of row i = D[i][pivot_j] for j < rank (zero beyond), so that
 * D = coeff . T.  ws: zx_gf2_workspace_bytes(m, n_cols) bytes.  Device
 * memory; asynchronous on s.  m <= 16384 (zx_gf2_eliminate's limit). */
zx_status zx_gf2_basis(const uint64_t* D, int32_t m, int32_t n_cols, int64_t ld, uint64_t* R,
                       int32_t* rank_dev, int32_t* pivot_cols_dev, uint64_t* coeff, int64_t ldc,
                       void* ws, size_t ws_bytes, hipStream_t s);
/* Per setting l (0 <= l < n_settings):
 *   omega^phase8 * sqrt(2)^pow_sqrt2 * prod_k h(k_alpha[k] pi/4, k_beta[k] pi/4; a_kl, b_kl)
 * with h(alpha, beta; a, b) = 1 + e^{i(alpha + a pi)} + e^{i(beta + b pi)}
 * - e^{i(alpha + beta + a pi + b pi)} (equation phase_pair) and a_kl, b_kl
 * bit l of row k of A and of B (n_terms x ld words, ld >= ceil(n_settings/64),
 * as written by zx_gf2_matmul).  Phases are multiples of pi/4 (integer codes,
 * as everywhere in this library).  Output per setting: mant[2l], mant[2l+1]
 * (real, imaginary; the larger magnitude in [0.5, 1), or both 0) and expo[l],
 * value = mant * 2^expo.  fp32 complex products, renormalised every 8 terms.
 * All arrays device memory.  Asynchronous on s. */
zx_status zx_phase_pair_product(const uint64_t* A, const uint64_t* B, int64_t ld, int32_t n_terms,
                                int64_t n_settings, const int8_t* k_alpha, const int8_t* k_beta,
                                int32_t phase8, int64_t pow_sqrt2, float* mant, int32_t* expo,
                                hipStream_t s);

/* ======================================================================
 * Generalised flow (the flow check before circuit extraction)
 *
 * The paper reduces diagrams by local complementation and pivoting and
 * eliminates binary matrices over F2 (detectors section, after equation
 * detector_sampling); circuit extraction and its flow check are the
 * standard procedures (Mhalla and Perdrix, ICALP 2008, for generalised
 * flow).  On the CURRENT diagram of each graph: output spiders form layer
 * 0; a spider u joins layer k when some set of processed spiders without an
 * input wire has odd neighbourhood, restricted to the spiders not yet
 * processed, equal to {u}; every layer is found by one Gauss-Jordan
 * elimination of those spiders' rows over F2 (its single-bit rows).
 * layers: sum of the graphs' n int32 (graph i's spiders after those of
 * graphs 0..i-1): the layer, or -1 for a spider that gets none or is not
 * present.  exists[i]: 1 if every present spider has a layer, 0 if not,
 * ZX_ECAPACITY for an arena the kernel does not take (layers unwritten).
 * Diagrams of up to 1024 spiders (ZX_ECAPACITY on the host otherwise).
 * ws: device workspace of zx_gflow_workspace_bytes(n_graphs), 256-byte
 * aligned; the call uploads the batch table into it and synchronises s
 * once before launching.  Device arrays; asynchronous on s after that.
 * ==================================================================== */
size_t zx_gflow_workspace_bytes(int32_t n_graphs);
zx_status zx_gflow(zx_graph* const* graphs, int32_t n_graphs, int32_t* layers, int32_t* exists, void* ws,
                   size_t ws_bytes, hipStream_t s);

/* ======================================================================
 * Circuit extraction
 *
 * The paper reduces diagrams and eliminates binary matrices over F2 but
 * leaves extraction to the standard procedure (Backens, Miller-Bakewell, de
 * Felice, Lobski, van de Wetering, "There and back again", Quantum 2021),
 * run here on the CURRENT diagram of each graph.  Every input spider is
 * first unfused into input -- a -H- b -H- v.  From the outputs inwards,
 * each round: Z rotations for the frontier spiders' phases (qubit order), CZ
 * gates for their mutual edges (pairs a < b in order), then Gauss-Jordan
 * elimination over F2 of the biadjacency between the frontier spiders that
 * are not input spiders (rows, qubit order) and their other neighbours
 * (columns, ascending id): lowest pivot column first, lowest row within
 * it, a row swap as three row additions, every row addition row_t += row_s
 * a CNOT with control t and target s, applied to the graph; then every row
 * with a single neighbour w is an H gate and that qubit's frontier moves to
 * w.  A Hadamard output wire is an H gate first.
 *
 * Gate q (uint32): type << 30 | a << 15 | b; types ZX_GATE_H (a = qubit),
 * ZX_GATE_RZ (a = qubit, b = k for diag(1, e^{i k pi/4})), ZX_GATE_CZ
 * (a < b), ZX_GATE_CNOT (a = control, b = target).  Gates closest to the
 * outputs come first: the diagram's map is G_1 G_2 ... G_m P up to a scalar,
 * where P takes input wire perm[q] to qubit q (after the Hadamards of
 * Hadamard input wires).
 * gates: n_graphs x max_gates (graph i's from i * max_gates); n_gates[i]:
 * gates of graph i's circuit (beyond max_gates only the first max_gates are
 * written, and status[i] = ZX_ECAPACITY); perm: sum of the graphs' n_out
 * int32 (graph i's after those of graphs 0..i-1), -1 for a qubit whose
 * frontier spider carries no input; status[i]: ZX_OK, ZX_ENOMATCH when the
 * procedure stops (no frontier row with a single neighbour, spiders left
 * outside the frontier, or a frontier spider without an input: the diagram
 * has no flow), ZX_ECAPACITY, or the diagram's own sticky status.
 * n + 2 n_in <= 1024 per graph (ZX_ECAPACITY on the host otherwise).
 * ws: device workspace of zx_extract_workspace_bytes(n_graphs), 256-byte
 * aligned; the call uploads the batch table into it and synchronises s
 * once before launching.  Device arrays; asynchronous on s after that.
 * ==================================================================== */
#define ZX_GATE_H 0u
#define ZX_GATE_RZ 1u
#define ZX_GATE_CZ 2u
#define ZX_GATE_CNOT 3u
size_t zx_extract_workspace_bytes(int32_t n_graphs);
zx_status zx_extract(zx_graph* const* graphs, int32_t n_graphs, int32_t max_gates, uint32_t* gates,
                     int32_t* n_gates, int32_t* perm, int32_t* status, void* ws, size_t ws_bytes,
                     hipStream_t s);

/* ======================================================================
 * Detector sampling: f = T e mod 2
 *
 * Section on the repetition-code example (equation detector_sampling) and
 * the detector paragraph after equation dets-only: column j of the binary
 * matrix T lists the detector/observable bits that error mechanism j flips;
 * mechanism j fires independently with probability prob[j].  As the paper
 * describes, the firing mechanisms of a shot are found by sampling the gap
 * to the next one from a geometric distribution (here for the largest
 * probability pmax, each mechanism so reached then firing with probability
 * prob[j] / pmax), so a shot costs O(pmax * n_err + 1).
 *
 * T as CSC: col_ptr[n_err + 1] (col_ptr[0] = 0, non-decreasing, col_ptr[n_err]
 * = nnz), col_idx[nnz] in [0, n_f).  Random numbers: SplitMix64, draw t of
 * shot s = mix64(seed + (s * 2^32 + t + 1) * 0x9E3779B97F4A7C15); per
 * candidate one draw u for the gap G = floor(ln U / ln(1 - pmax)),
 * U = ((u >> 11) + 1) * 2^-53 (none when pmax = 1), then one draw v: fires
 * iff (v >> 11) < floor(prob[j] / pmax * 2^53), all in fp64.  Shot s
 * depends only on (seed, s), so ranges of shots can be sampled separately.
 * out: n_shots x ld_out words (ld_out >= ceil(n_f/64)); row i = shot
 * shot0 + i.  n_f <= 2048, shot0 + n_shots <= 2^31.  ws: device workspace of
 * zx_detector_workspace_bytes(n_err), 256-byte aligned.  A model that fails
 * validation on the device (probabilities outside [0, 1], bad col_ptr or
 * col_idx) sets the workspace status to ZX_EINVAL (zx_detector_status) and
 * the output rows are all zero.  Device arrays; asynchronous on s.
 * ==================================================================== */
size_t zx_detector_workspace_bytes(int32_t n_err);
zx_status zx_detector_sample(const int32_t* col_ptr, const int32_t* col_idx, int64_t nnz, const double* prob,
                             int32_t n_err, int32_t n_f, uint64_t seed, int64_t shot0, int64_t n_shots,
                             uint64_t* out, int64_t ld_out, void* ws, size_t ws_bytes, hipStream_t s);
/* Status of the last sampling call that used ws (synchronises s). */
zx_status zx_detector_status(const void* ws, hipStream_t s);

/* ======================================================================
 * Learned rewrite proposal: scoring network, training kernels, rollouts
 *
 * The paper fixes no proposal policy; this one ranks the candidates of a
 * round.  Network: score = w2 . relu(W1^T x + b1) + b2, x of ZX_MLP_IN
 * features, ZX_MLP_HID hidden units.  x, W1 and w2 enter every product
 * rounded to bf16 (round to nearest even); sums are fp32.  The parameters
 * live in caller memory (device):
 *   param  fp32 master, ZX_MLP_NPARAM floats: W1[ZX_MLP_IN][ZX_MLP_HID]
 *          (input major) | b1[ZX_MLP_HID] | w2[ZX_MLP_HID] | b2
 *   wbf16  bf16 copies used by the kernels, ZX_MLP_NBF16 halves: W1
 *          transposed (hidden unit major) | w2.  zx_mlp_sync refreshes it.
 * ==================================================================== */
#define ZX_MLP_IN 16
#define ZX_MLP_HID 256
#define ZX_MLP_NPARAM (ZX_MLP_IN * ZX_MLP_HID + 2 * ZX_MLP_HID + 1)
#define ZX_MLP_NBF16 (ZX_MLP_IN * ZX_MLP_HID + ZX_MLP_HID)

struct zx_mlp {
  float* param;
  uint16_t* wbf16;
};

/* wbf16 <- bf16(param). */
zx_status zx_mlp_sync(const zx_mlp* w, hipStream_t s);
/* score[r] for rows r of x (rows x ZX_MLP_IN bf16, row major). */
zx_status zx_mlp_forward(const zx_mlp* w, const uint16_t* x, int64_t rows, float* score,
                         hipStream_t s);
/* Softmax cross-entropy per segment: rows seg_off[i] .. seg_off[i+1]-1 are
 * the candidates of state i; rows with cost < 0 are absent.  Target = even
 * over the t present rows of least cost.  loss[i] = logsumexp - (sum of the
 * targets' scores) / t (0 for a segment with no present row); dscore =
 * (softmax - target) / n_seg on present rows, 0 elsewhere. */
zx_status zx_mlp_loss(const float* score, const int64_t* cost, const int32_t* seg_off,
                      int32_t n_seg, float* dscore, float* loss, hipStream_t s);
/* grad (ZX_MLP_NPARAM floats, overwritten) = d(sum_r dscore[r] score[r]) /
 * d(param), treating the bf16 rounding of W1 and w2 as the identity.  The
 * sums over rows are reduced in a fixed order (deterministic). */
size_t zx_mlp_workspace_bytes(int64_t rows);
zx_status zx_mlp_backward(const zx_mlp* w, const uint16_t* x, const float* dscore, int64_t rows,
                          float* grad, void* ws, size_t ws_bytes, hipStream_t s);
/* Adam on the fp32 master (m, v: ZX_MLP_NPARAM floats each), then wbf16
 * refresh.  step counts from 1; bias corrections 1 - beta^step. */
zx_status zx_mlp_adam(const zx_mlp* w, const float* grad, float* m, float* v, float lr,
                      float beta1, float beta2, float eps, int32_t step, hipStream_t s);

/* The learned proposal's view of one diagram state (its CURRENT section):
 * the candidates of the next round as the learned schedule lists them (LC
 * candidates ascending while there are any, else the pivot edges), and for
 * each the ZX_MLP_IN bf16 features the learned simplification scores
 * (listed under zx_rollout).  Writes the count to *n_cand (one device int32)
 * and the first min(count, max_cand) candidates and feature rows to cand
 * (two int32 each: u, v; v = -1 for an LC candidate) and feats (row-major,
 * ZX_MLP_IN per row), all device memory of the caller.
 * ZX_ECAPACITY when the diagram does not fit the kernel's LDS (about 1000
 * spiders).  Asynchronous on s; the arena is only read.  The paper leaves the
 * proposal's inputs open: these are the features of this library's
 * network. */
zx_status zx_policy_features(const zx_graph* g, int32_t* cand, uint16_t* feats, int32_t max_cand,
                             int32_t* n_cand, hipStream_t s);

/* Rollouts for training labels.  Item i = (state i / per_state, slot
 * k = i % per_state) on states[i / per_state] (CURRENT diagrams, read only;
 * at most 1024 spiders).  The kernel lists the state's candidates as the
 * learned schedule does (LC candidates ascending while there are any, else
 * the pivot edges), takes candidate c = k (all of them when there are at
 * most per_state, else c = floor(k * count / per_state)), writes its
 * features, applies it, runs the greedy schedule to the fixed point and
 * reduces the output frontier:
 *   cost[i]   = Hadamard edges left + frontier row additions (-1: no such
 *               candidate, also for a state at its fixed point; -3: the
 *               state is too large; -4: the round bound was exceeded)
 *   fill[i]   = edges toggled on from the state to the end
 *   move[i]   = {0 (LC), u, -1} or {1 (pivot), u, v}, or {-1, -1, -1}
 *               without a candidate
 *   feats[i]  = ZX_MLP_IN bf16 features of the candidate: for endpoint u,
 *     degree / N, phase class one-hot {k = 0 mod 4, k = 2 mod 4, k odd},
 *     boundary-attached neighbours / N, two-hop count / N (spiders at
 *     distance exactly 2), Pauli neighbours / N (k = 0 mod 4); the same
 *     seven for v (zeros for an LC candidate); rule bit (1: pivot);
 *     constant 1.  N = present spiders; quotients in fp32, then bf16.
 * Synchronous (uploads the state table into ws). */
size_t zx_rollout_workspace_bytes(zx_graph* const* states, int32_t n_states);
zx_status zx_rollout(zx_graph* const* states, int32_t n_states, int32_t per_state, int64_t* cost,
                     int64_t* fill, int32_t* move, uint16_t* feats, void* ws, size_t ws_bytes,
                     hipStream_t s);

/* ======================================================================
 * Serving: continuous batching of simplification requests
 *
 * The paper's compile-once / sample-many use (section "Complexity",
 * paragraph "Compilation") makes simplification a per-circuit service.  A
 * server owns a caller-provided device pool; every request gets a slice of
 * it (its arena) from submit until its result is harvested.  Submit uploads
 * the request and appends it to a ring in coherent host memory; a resident
 * kernel (two 512-thread workgroups per CU) claims ring entries in order,
 * one workgroup per diagram, and posts each summary and a completion flag
 * back to host memory, so no request waits for another to finish.  The
 * kernel leaves after 50 ms without work; submit and poll start it again
 * when requests are waiting.  zx_server_poll harvests completions (results
 * out, slices freed).  Calls on one server must not overlap (one thread at
 * a time); different servers are independent.
 * ==================================================================== */
typedef struct zx_server zx_server;

typedef struct {
  int32_t n, n_in, n_out, pad;  /* spiders, input and output wires */
  const uint64_t* adj;          /* host, n x ceil(n/64) words, symmetric */
  const int8_t* phase;          /* host, n entries in 0..7 (units of pi/4) */
  const int32_t* inputs;        /* host, spider of input wire i */
  const int32_t* outputs;       /* host, spider of output wire j */
  const uint8_t* bnd_is_h;      /* host or NULL */
  int64_t tag;                  /* returned unchanged */
} zx_request;

typedef struct {
  int64_t ticket, tag;
  int32_t status;               /* sticky status of the request's diagram */
  int32_t n_alive, rounds, n_trace, rank, phase8;
  int64_t n_edges, rowops, pow_sqrt2, fill_in;
  int32_t policy;               /* schedule of the result (ZX_POLICY_*) */
  int32_t pad;
  double t_submit, t_launch, t_done;  /* host steady clock, seconds: submission,
                                         start on the device, result seen by poll */
  double t_device;              /* seconds from a workgroup claiming the request
                                   to its result written (device clock) */
  double t_claim_dev, t_end_dev;  /* the two device-clock instants, seconds */
} zx_result;

typedef struct {
  int64_t submitted, refused, completed, batches, pending, running;
  size_t pool_bytes, pool_used, pool_peak;
} zx_server_stats;

#define ZX_SERVE_TRUSTED 0x1u  /* submit skips the O(n^2) symmetry test */

/* pool: device memory owned by the caller (256-byte aligned) that the server
 * uses for a 256-byte control block and the request arenas.  max_batch is
 * kept for compatibility (the ring holds 65536 requests).  o: policy and
 * extract and flags (ZX_FALLBACK; tune_id and max_rounds are ignored); NULL
 * = greedy with extraction.  Requests up to 8192 spiders (4096 with the
 * learned policy without ZX_FALLBACK; with it, larger requests run greedy). */
zx_status zx_server_create(zx_server** sv, void* pool, size_t pool_bytes, int32_t max_batch,
                           const zx_simplify_opts* o, uint32_t flags);
/* Validate and upload a request (synchronous for the host arrays).
 * ZX_EBUSY: the pool or the ring has no room now (admission refused; retry
 * after polling).  ZX_ECAPACITY: the request can never be served. */
zx_status zx_server_submit(zx_server* sv, const zx_request* r, int64_t* ticket);
/* Make progress and return up to max finished results. */
zx_status zx_server_poll(zx_server* sv, zx_result* out, int32_t max, int32_t* n_out);
zx_status zx_server_stats_read(const zx_server* sv, zx_server_stats* st);
/* Lets the resident kernel finish the submitted requests and stop, then
 * frees the server (not the pool).  Results not yet polled are dropped. */
void zx_server_destroy(zx_server* sv);

#ifdef __cplusplus
}
#endif
#endif /* ZX_H */
