/*
 * qs.h -- C ABI of the MI355X structured-layer state-vector library (libqs.so).
 *
 * The library applies gate streams to a 2^n complex state vector held in device
 * memory.  Its fused path rewrites a stream into structured layers, exactly in
 * exact arithmetic (paper, Section "Hand-Tuned Metal Shaders": "Kernel Taxonomy"
 * and "Semantics-Preserving Fusion"):
 *   - diagonal runs (Z-type rotations, CZ/CPHASE, ZZ couplings, multi-controlled
 *     phases) become one phase-lookup-table pass, bonds grouped by equal angle
 *     with tables built in double precision;
 *   - X/CNOT/SWAP runs become one GF(2)-affine index-permutation gather;
 *   - windows of single-qubit gates collapse per wire into one 2x2 product
 *     (complex128) and run as tensor-product tile passes;
 *   - QFT stages (H plus its controlled-phase ladder) become butterfly-plus-
 *     twiddle operations, several stages per pass;
 *   - Hadamard layers become Walsh-Hadamard butterflies;
 *   - same-family XX / YY runs are conjugated into the diagonal machinery;
 *   - dense k-qubit gates, and windows of decomposed gates with no cheaper
 *     structure, run as dense blocks on the matrix cores.
 * The plain path applies one kernel per gate (the paper's per-gate pure tier,
 * Appendix A).  Reductions (norms, overlaps, Pauli expectations, gradients) are
 * accumulated in FP64 with compensated sums.
 *
 * Conventions
 *   - Qubit q is bit n-1-q of the basis index (MSB-first), everywhere.
 *   - Amplitudes are interleaved (re, im): float pairs for QS_C64, double pairs
 *     for QS_C128; a state of n qubits occupies 2^n amplitudes.
 *   - Pauli masks (qs_pauli) and multi-controlled masks (qs_gate.mask) use
 *     qubit numbering: bit q refers to qubit q.
 *   - Every call returns a qs_status; on failure nothing has been applied or
 *     written (validation happens before any device work), and
 *     qs_last_error() gives a message for the calling thread.
 *   - Device work is enqueued on the state's HIP stream.  Calls that return
 *     host values (expectations, norms, gradients, infidelity) synchronise that
 *     stream; asynchronous device faults surface there as QS_EDEVICE.
 *
 * Ownership
 *   - Host arrays passed in (gates, matrices, Pauli terms, parameters) are read
 *     only during the call; output arrays are written only during the call.
 *   - A device buffer given to qs_alloc is borrowed: it must outlive the state
 *     and is never freed by the library.  Buffers the library allocates are
 *     freed by qs_free.
 *   - Plans own their device-side tables (LUTs, matrices, masks); a plan can be
 *     applied to any state of the same qubit count and dtype, but a plan and a
 *     state must not be used from two threads at once.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QS_OK = 0,
  QS_EINVAL = -1,       /* invalid argument: wires, sizes, counts, mismatch */
  QS_ENOMEM = -2,       /* capacity exceeded or device allocation failed */
  QS_EDEVICE = -3,      /* HIP runtime / kernel error */
  QS_EUNSUPPORTED = -4  /* valid request the library does not implement */
} qs_status;

typedef enum { QS_C64 = 0, QS_C128 = 1 } qs_dtype;

#define QS_MAX_QUBITS 32
#define QS_MAX_GATE_WIRES 6

/* Gate kinds.  Matrices (c = cos(theta/2), s = sin(theta/2)):
 *   H, X, Y, Z, S = diag(1, i), SDG, T = diag(1, e^{i pi/4}), TDG,
 *   SX = [[1+i, 1-i], [1-i, 1+i]] / 2,
 *   RX = exp(-i theta X/2), RY = exp(-i theta Y/2), RZ = exp(-i theta Z/2),
 *   P = diag(1, e^{i theta}), U = arbitrary 2x2 given in mat,
 *   CNOT(control, target), CZ, CPHASE = diag(1, 1, 1, e^{i theta}), SWAP,
 *   RZZ / RXX / RYY = exp(-i theta P(x)P / 2),
 *   CU(control, target) = controlled version of the 2x2 in mat,
 *   MCZ / MCP = phase -1 / e^{i theta} on the basis states where every qubit
 *   of gate.mask is 1,
 *   UNITARY = arbitrary 2^nw x 2^nw matrix on wires[0..nw-1] (wires[0] is the
 *   most significant row bit), nw <= QS_MAX_GATE_WIRES. */
typedef enum {
  QS_GATE_I = 0, QS_GATE_H, QS_GATE_X, QS_GATE_Y, QS_GATE_Z, QS_GATE_S, QS_GATE_SDG,
  QS_GATE_T, QS_GATE_TDG, QS_GATE_SX, QS_GATE_RX, QS_GATE_RY, QS_GATE_RZ, QS_GATE_P,
  QS_GATE_U, QS_GATE_CNOT, QS_GATE_CZ, QS_GATE_CPHASE, QS_GATE_SWAP, QS_GATE_RZZ,
  QS_GATE_RXX, QS_GATE_RYY, QS_GATE_CU, QS_GATE_MCZ, QS_GATE_MCP, QS_GATE_UNITARY,
  QS_GATE_KIND_COUNT
} qs_gate_kind;

/* One gate.  Angle = theta when param < 0, else theta + scale * params[param]
 * (parameters are bound with qs_plan_set_params / the params argument of
 * qs_apply_gates).  mat: interleaved complex128, row-major, for U, CU (2x2)
 * and UNITARY (2^nw x 2^nw); NULL otherwise. */
typedef struct {
  int32_t kind;
  int32_t nw;
  int32_t wires[QS_MAX_GATE_WIRES];
  int32_t param;
  int32_t reserved;
  double theta;
  double scale;
  uint64_t mask;
  const double* mat;
} qs_gate;

/* A Pauli term coeff * P, P = prod over qubits of X (x bit), Z (z bit) or
 * Y (both bits); bit q = qubit q. */
typedef struct {
  double coeff;
  uint64_t x_mask;
  uint64_t z_mask;
} qs_pauli;

typedef enum { QS_PLAIN = 0, QS_FUSED = 1 } qs_mode;

/* Plan options; pass NULL for defaults (QS_FUSED, tile/round sizes from the
 * library's tuned table). */
typedef struct {
  int32_t mode;             /* QS_PLAIN: one layer per gate; QS_FUSED: detectors on */
  int32_t max_tile_bits;    /* 0 = default; amplitudes per tile pass = 2^max_tile_bits */
  int32_t dense_k_max;      /* 0 = default (6); largest UNITARY gate run as a dense block */
  int32_t window_k;         /* dense-window fusion (generic matrix fusion of decomposed
                               blocks, Section "Limitations and Future Work"): 0 = default
                               (5), 4..6 = largest window, -1 = off.  Consecutive constant
                               gates are collected into windows of at most window_k qubits;
                               the window plan is used when it needs fewer passes than the
                               structured plan. */
  int32_t low_bits;         /* contiguous low state bits of a tile pass over high bits
                               (runs of 2^low_bits amplitudes in HBM): 0 = per group, the
                               tile's remaining bits (at least 4); 2..8 = fixed */
  int32_t coset_order;      /* which coset of its tile bits each workgroup of a tile pass
                               takes: 0 = by geometry (contiguous tiles and tiles with runs
                               of at most 16 amplitudes XCD-blocked, longer runs in launch
                               order), 1 = XCD-blocked (each of the 8 XCDs a contiguous
                               range of cosets), 2 = launch order (the workgroups resident
                               at one time, on all XCDs, take neighbouring cosets) */
  int32_t diag_low_bits;    /* tile passes over high bits that carry diagonal layers:
                               0 = default, -1 = the same low bits as other passes,
                               2..8 = at most this many low bits (smaller tiles) */
  int32_t balance_passes;   /* 0 = default: single-qubit ops after a tile pass's last
                               diagonal layer move to the next tile pass when that
                               evens out the two passes' arithmetic; -1 = off */
} qs_plan_opts;

typedef struct qs_state qs_state;
typedef struct qs_plan qs_plan;
typedef struct qs_batch qs_batch;

/* ---- library ------------------------------------------------------------ */

/* Message for the calling thread's last non-OK status (never NULL). */
const char* qs_last_error(void);
/* Version string and the device architecture the library was built for. */
const char* qs_version(void);
/* Device bytes the library holds in amplitude buffers it allocated (states,
 * scratch halves, adjoint work states and scratch, batch arenas), and the cap
 * on them: the environment variable QS_MAX_BYTES (bytes, read at the first
 * allocation; unset or 0: no cap).  An allocation that would exceed the cap
 * fails with QS_ENOMEM before any device call.  Either pointer may be NULL. */
qs_status qs_memory_info(size_t* held, size_t* cap);

/* ---- states (Section "State Management": a flat amplitude array) ------- */

/* Create a state of n qubits (1 <= n <= QS_MAX_QUBITS) on the current HIP
 * device.  buf / scratch: device buffers of at least 2^n amplitudes each, or
 * NULL to let the library allocate.  The scratch buffer is the second half of
 * the out-of-place permutation gather's ping-pong; it is only allocated when
 * such a layer first runs if NULL is passed.  bytes: capacity of each given
 * buffer (ignored for NULL buffers).  stream: hipStream_t or NULL for the
 * null stream.  The amplitudes are left uninitialised.  QS_ENOMEM when the
 * request exceeds the device's free memory (checked before allocating). */
qs_status qs_alloc(int n, qs_dtype dtype, void* buf, void* scratch, size_t bytes,
                   void* stream, qs_state** out);
qs_status qs_free(qs_state* s);
/* Current amplitude buffer (it alternates between buf and scratch after
 * permutation layers) and the other buffer (NULL until allocated). */
qs_status qs_state_buffers(const qs_state* s, void** current, void** other);
qs_status qs_state_info(const qs_state* s, int* n, int* dtype);

/* |index> (index in the MSB-first convention, index < 2^n). */
qs_status qs_set_basis(qs_state* s, uint64_t index);
/* |+>^n: every amplitude 2^{-n/2}. */
qs_status qs_set_uniform(qs_state* s);
/* Copy 2^n host amplitudes of the state's dtype into the state (sync). */
qs_status qs_upload(qs_state* s, const void* host, size_t bytes);
/* Copy the state into a host array of 2^n amplitudes (sync). */
qs_status qs_download(const qs_state* s, void* host, size_t bytes);
/* dst <- src (same n; dtypes may differ: converted on the device). */
qs_status qs_copy(qs_state* dst, const qs_state* src);
/* Wait for the state's stream; reports asynchronous faults as QS_EDEVICE. */
qs_status qs_sync(qs_state* s);

/* ---- plans (Section "Semantics-Preserving Fusion") --------------------- */

/* Validate a gate stream and build its layer plan (host only; no device work
 * until the plan is first applied).  n_params: length of the parameter vector
 * the stream refers to (every gate's param must be < n_params).  Invalid,
 * duplicate or out-of-range wires, a kind/arity mismatch or a missing matrix
 * give QS_EINVAL. */
qs_status qs_plan_create(int n, const qs_gate* gates, size_t n_gates, size_t n_params,
                         const qs_plan_opts* opts, qs_plan** out);
/* Bind parameter values (re-computes LUTs, matrices and twiddles; the layer
 * structure is unchanged).  Must be called before the first apply when
 * n_params > 0. */
qs_status qs_plan_set_params(qs_plan* p, const double* params, size_t n_params);
qs_status qs_plan_num_layers(const qs_plan* p, size_t* out);
/* JSON description of the layers (kinds, bits, passes, tables) for tests and
 * tooling.  Writes at most cap bytes (NUL-terminated); *needed receives the
 * full length + 1. */
qs_status qs_plan_describe(const qs_plan* p, char* buf, size_t cap, size_t* needed);
qs_status qs_plan_free(qs_plan* p);
/* A new plan applying the inverse of p (layers in reverse order, each layer
 * inverted: U^dagger windows, inverse QFT stages, conjugated phase tables,
 * inverse permutation), sharing p's current parameter values; free it with
 * qs_plan_free.  Used by the adjoint sweep; also usable to un-compute. */
qs_status qs_plan_inverse(const qs_plan* p, qs_plan** out);

/* Apply layers [first, first + count) of a plan to a state (asynchronous, on
 * the state's stream).  count = (size_t)-1 applies through the last layer.
 * (Section "Hand-Tuned Metal Shaders": each fused layer is one kernel of the
 * "Kernel Taxonomy"; the rewrite is the "Semantics-Preserving Fusion" one, so
 * the result equals the gate-by-gate product up to rounding.)  QS_EINVAL when
 * the plan's and the state's qubit counts differ or a parametrised plan has
 * no bound parameters; nothing is applied then. */
qs_status qs_apply_layer(qs_state* s, const qs_plan* p, size_t first, size_t count);
/* Apply every layer of a plan through one HIP graph launch (asynchronous, on
 * the state's stream).  The plan's layer sequence is recorded as a graph on
 * the first call for this state, plan and parameter values (and for the
 * buffer the state currently starts from), then replayed: for small states
 * the per-layer launch cost disappears.  Up to 8 graphs are kept per state
 * (freed with it); new parameters (qs_plan_set_params) record a new graph.
 * Plans containing plain gates on 3 or more qubits run as qs_apply_layer. */
qs_status qs_apply_graph(qs_state* s, const qs_plan* p);
/* Apply every layer of a plan, then write ||psi||^2 of the result (FP64) to
 * *norm2 (host; the call waits for the device).  When the plan ends in a
 * tile pass or a GF(2) gather, that kernel sums |psi|^2 over the amplitudes
 * it writes, in a fixed order, so the norm costs no extra read of the state;
 * otherwise a separate reduction runs (the same value as qs_norm2 up to the
 * order of the FP64 sums).  Allocates a small per-state partials buffer on
 * first use (8 bytes per tile, or per wavefront of a gather, of the last
 * layer). */
qs_status qs_apply_norm2(qs_state* s, const qs_plan* p, double* norm2);
/* Plain per-gate path: one kernel per gate, no fusion (the baseline).  This
 * is the paper's structured per-gate tier (Section "Same-Machine External
 * Baselines": diagonal gates as broadcast phase multiplies, controlled
 * single-qubit gates as half-state updates, SWAP as a permutation; Appendix
 * "Pure MLX versus a Hand-Written Kernel", "The pure-MLX path": a single-qubit
 * gate as the (A, 2, B) pair update).  gates / params: host arrays read during
 * the call; every gate is validated before the first launch (QS_EINVAL). */
qs_status qs_apply_gates(qs_state* s, const qs_gate* gates, size_t n_gates,
                         const double* params, size_t n_params);

/* ---- reductions (FP64, compensated, deterministic) --------------------- */
/* Section "State Management" (normalisation, probabilities and expectation
 * values of Pauli observables) and Section "Independent complex128
 * validation" (norm drift and infidelity against a reference).  Each
 * amplitude is widened to FP64 and summed with Neumaier compensation per
 * thread, then in a fixed order over threads and workgroups, so the results
 * are bitwise repeatable.  They synchronise the state's stream. */

/* sum_t coeff_t <psi|P_t|psi> (host terms[n_terms], read during the call);
 * per_term (nullable, host, n_terms doubles) receives each term's
 * <psi|P_t|psi> times coeff_t, total (host) the sum.  Not normalised by
 * ||psi||^2. */
qs_status qs_expect(qs_state* s, const qs_pauli* terms, size_t n_terms,
                    double* per_term, double* total);
qs_status qs_norm2(qs_state* s, double* out);
/* <a|b> (a conjugated) as out[0] + i out[1]; a and b may differ in dtype. */
qs_status qs_overlap(qs_state* a, qs_state* b, double out[2]);
/* 1 - |<a|b>|^2 / (|a|^2 |b|^2), evaluated without cancellation as
 * D (1 - D/4) with D = || b/|b| - e^{i arg<a|b>} a/|a| ||^2. */
qs_status qs_infidelity(qs_state* a, qs_state* b, double* out);
/* Gather the amplitudes at the given indices (MSB-first, each < 2^n) into
 * host_amps (count amplitudes of the state's dtype, interleaved; sync). */
qs_status qs_amplitudes(qs_state* s, const uint64_t* idx, size_t count, void* host_amps);

/* ---- read-out (paper, Sections "State Management" and "Algorithm
 * Implementations": measurement and sampling from the state) ------------- */
/* Shot sampling of p_i = |psi_i|^2 / ||psi||^2.  For each caller-provided
 * uniform number u[k] in [0, 1) (host, count of them), out[k] (host) receives
 * the first index i whose cumulative mass sum_{j<=i} |psi_j|^2 exceeds
 * u[k] ||psi||^2; the cumulative sums are FP64 with a fixed summation order,
 * so equal inputs give equal draws.  A drawn index always has p_i > 0.
 * QS_EINVAL for u outside [0, 1) or a state without mass (nothing is drawn). */
qs_status qs_sample(qs_state* s, const double* u, size_t count, uint64_t* out);
/* qs_sample without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same draws, bit for bit, with the norm reduction's partials,
 * the cumulative sums and the staged uniforms and indices held in a static
 * device array of the library (about 9.6 MB per GPU, kept until the process
 * ends; looked up once per device on the first call there).  u and out are
 * host arrays of count entries, as for qs_sample.  Limits: at most 26 qubits
 * and at most 65536 draws per call; larger requests give QS_EINVAL before any
 * device work.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (concurrent threads or streams) race and must be
 * serialised by the caller. */
qs_status qs_sample_noalloc(qs_state* s, const double* u, size_t count, uint64_t* out);
/* Marginal distribution (unnormalised: sums of |psi_i|^2, FP64) over the
 * qubits set in qubit_mask (bit q = qubit q, at most 16 of them) into out
 * (host, 2^k doubles).  Bin index: the selected qubits read as a sub-register,
 * the lowest-numbered selected qubit most significant (MSB-first). */
qs_status qs_marginal(qs_state* s, uint64_t qubit_mask, double* out);

/* ---- adjoint gradients -------------------------------------------------- */
/* The adjoint method is this library's addition.  The paper differentiates
 * its variational ansatz by parameter shift (Section "Algorithm
 * Implementations": parameter-shift gradients with Adam), which costs two
 * circuits per parameter (Section "Detailed Algorithm Performance", the
 * ansatz scaling table, which names automatic differentiation as the way to
 * extend that range).  This call returns the same gradient, exact up to
 * rounding, from one forward and one backward sweep. */

/* Energy E = <psi_L|H|psi_L> and dE/dparams of the plan applied to the given
 * state (in: initial state; out: the final state psi_L).  Uses the adjoint
 * method: lambda = H psi_L, then the fused layers are un-applied from psi and
 * lambda together, accumulating 2 Re <lambda| dU psi> per parameter in FP64.
 * grad has n_params entries (must equal the plan's).  Parameters may appear in
 * RX, RY, RZ and P gates of single-qubit windows and in diagonal gates (RZ, P,
 * CPHASE, RZZ, MCP); a parameter on any other kind gives QS_EUNSUPPORTED.
 * Memory: the first call allocates two work states of psi's size (each with
 * its own gather scratch when the plan has permutation layers) and a small
 * device scratch area; they stay with psi for later calls and are released
 * by qs_free(psi).  QS_ENOMEM when they do not fit. */
qs_status qs_adjoint_grad(qs_state* psi, const qs_plan* p, const qs_pauli* terms,
                          size_t n_terms, double* energy, double* grad, size_t n_params);

/* ---- batches of circuits (many states, one graph launch) ---------------- */
/* Batching is this library's addition for the launch-bound regime the paper
 * reports (Section "Background", "GPU Acceleration Paradigms": gate batching
 * to amortise overhead; Section "Limitations and Future Work" and the
 * QASM sweep of Appendix "Complete Per-Workload Speedups": below ~15 qubits
 * a circuit sits at kernel-launch overhead).  The instances are typically the
 * QAOA ansatz of Section "Algorithm Implementations" (cost layer
 * e^{-i gamma H_C}, mixer e^{-i beta H_M}, from |+>^n) on different graphs,
 * sizes and angles. */

/* A batch owns n_inst states (qubit counts n_qubits[i], one device arena) and
 * one plan per instance (plans[i], borrowed, must outlive the batch, all with
 * mode QS_FUSED and the same dtype).  Every instance starts from |+>^n (init =
 * 1) or |0...0> (init = 0).  The whole layer sequence of all instances is
 * recorded once as a HIP graph on the given stream. */
qs_status qs_batch_create(size_t n_inst, const int* n_qubits, const qs_plan* const* plans,
                          int init, qs_dtype dtype, void* stream, qs_batch** out);
/* Re-read every plan's bound parameters (call after qs_plan_set_params). */
qs_status qs_batch_refresh(qs_batch* b);
/* One graph launch: initialise all instances and apply all their layers. */
qs_status qs_batch_run(qs_batch* b);
/* Expectation of a diagonal observable per instance (terms with x_mask = 0
 * only): obs[i] has n_terms[i] terms; out receives n_inst values (sync). */
qs_status qs_batch_expect_diag(qs_batch* b, const qs_pauli* const* obs,
                               const size_t* n_terms, double* out);
/* Stores diagonal observables (as for qs_batch_expect_diag) on the device
 * once, for loops that re-run the batch with new parameters and read the
 * same observables each time; replaces any stored before.  Terms are read
 * during the call only.  (Section "Algorithm Implementations": the QAOA
 * cost expectation per instance.) */
qs_status qs_batch_set_observables(qs_batch* b, const qs_pauli* const* obs, const size_t* n_terms);
/* Expectation of the stored observables per instance, as qs_batch_expect_diag
 * (sync); QS_EINVAL when none are stored. */
qs_status qs_batch_expect_stored(qs_batch* b, double* out);
/* Expectation of any Pauli sum per instance (sync): Z-type terms of all
 * instances in one batched FP64 reduction, terms with X or Y factors per
 * instance with pair reads.  obs[i] has n_terms[i] terms; out receives n_inst
 * values. */
qs_status qs_batch_expect(qs_batch* b, const qs_pauli* const* obs, const size_t* n_terms, double* out);
/* State of instance i as a view (valid until the batch is freed). */
qs_status qs_batch_state(qs_batch* b, size_t i, qs_state** view);
qs_status qs_batch_free(qs_batch* b);

/* ---- instrumentation ----------------------------------------------------- */

/* When enabled, every kernel the library launches on a state's stream is
 * bracketed by HIP events and its duration is accumulated per kernel name. */
qs_status qs_profile_enable(int on);
/* Kernel statistics since the last reset, as JSON
 * [{"kernel": name, "launches": k, "total_ms": t}, ...] (sync). */
qs_status qs_profile_report(char* buf, size_t cap, size_t* needed);
qs_status qs_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
