/*
 * hhlsv.h -- C ABI of libhhlsv, an MI355X (gfx950) state-vector simulator
 * for the HHL quantum linear solver.
 *
 * The calls follow the problem statement of Zheng et al., "Early
 * Exploration of a Flexible Framework for Efficient Quantum Linear Solvers in
 * Power Systems" (PESGM 2024), Sec. III-A "Practical HHL procedures": given
 * A and b of A x = b, build the HHL circuit (step 2, Fig. 5), run it on a
 * state-vector simulator whose dominant cost is the unitary evolution of the
 * state (Sec. II-C), read the state vector (step 3) and recover x (step 4).
 * Gate fusion (Sec. II-C, Fig. 4) is exposed as fuse().
 *
 * Conventions
 *   - Qubit q is bit q of the amplitude index (little-endian).
 *   - An n-qubit state is 2^n complex amplitudes, interleaved (re, im):
 *     SV_C128 = two doubles per amplitude (16 B), SV_C64 = two floats (8 B).
 *   - A k-qubit matrix on the qubit list (q_0..q_{k-1}) is row-major
 *     2^k x 2^k complex (interleaved doubles); its row/column index is
 *     r = sum_l bit(q_l) 2^l.
 *   - HHL register layout: system qubits 0..ns-1, clock qubits ns..ns+m-1
 *     (clock bit j is qubit ns+j), ancilla ns+m; n = ns + m + 1.
 *
 * Errors: every call returns an sv_status; on failure sv_last_error() gives
 * a thread-local message.  No call aborts or throws across the ABI.  Inputs
 * are validated before any device work.  HIP errors are reported as
 * SV_ERR_HIP; a kernel fault leaves the HIP context unusable (sticky), so the
 * caller must treat SV_ERR_HIP as fatal for the process's GPU work.
 *
 * Ownership: inputs are copied at the call and stay the caller's.  The
 * library owns sv_state / sv_circuit / svb / svs objects until their destroy
 * or stop call; sv_create_from_buffer adopts memory the caller keeps alive.
 * Outputs go to caller-allocated buffers.
 *
 * Streams: device work is ordered on the state's stream (default: a stream
 * the library creates per state).  sv_apply is asynchronous; calls that
 * return host data synchronise that stream.  A state is used by one thread
 * at a time; circuits are read-only after construction and may be shared.
 */
#ifndef HHLSV_H
#define HHLSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SV_OK = 0,
    SV_PENDING = 1,
    SV_ERR_INVALID = -1,
    SV_ERR_OOM = -2,
    SV_ERR_HIP = -3,
    SV_ERR_NOT_SYMMETRIC = -4,
    SV_ERR_NOT_POSDEF = -5,
    SV_ERR_SHAPE = -6,
    SV_ERR_BUSY = -7,
    SV_ERR_SINGULAR = -8     /* b reaches a zero eigenvalue (signed HHL)  */
} sv_status;

typedef enum { SV_C128 = 0, SV_C64 = 1 } sv_dtype;

/* Gate kinds for circuit_add_gate (textbook / OpenQASM definitions). */
typedef enum {
    SV_GATE_H = 0,      /* qubits (q)                                     */
    SV_GATE_X = 1,      /* qubits (q)                                     */
    SV_GATE_RY = 2,     /* qubits (q); params (theta): [[c,-s],[s,c]]     */
    SV_GATE_RZ = 3,     /* qubits (q); params (theta):
                           diag(e^{-i theta/2}, e^{i theta/2})            */
    SV_GATE_P = 4,      /* qubits (q); params (phi): diag(1, e^{i phi})   */
    SV_GATE_U3 = 5,     /* qubits (q); params (theta, phi, lambda)        */
    SV_GATE_CX = 6,     /* qubits (control, target)                       */
    SV_GATE_CP = 7,     /* qubits (a, b); params (phi): e^{i phi} on |11> */
    SV_GATE_SWAP = 8,   /* qubits (a, b)                                  */
    SV_GATE_DENSE = 9,  /* qubits (q_0..q_{k-1}), k <= 12; params: the
                           2^k x 2^k matrix (2 * 4^k doubles)             */
    SV_GATE_CDENSE = 10,/* qubits (c, q_0..q_{k-1}): DENSE applied where
                           bit c is 1                                     */
    SV_GATE_UCRY = 11,  /* qubits (t, c_0..c_{r-1}), r <= 20; params: 2^r
                           angles; RY(angle[v]) on t where v = sum_l
                           bit(c_l) 2^l                                   */
    SV_GATE_DIAG = 12,  /* qubits (q_0..q_{k-1}), k <= 12; params: 2^k
                           complex diagonal entries (2 * 2^k doubles)     */
    SV_GATE_MUX2 = 13,  /* qubits (c_0, c_1, q_0..q_{k-1}), k <= 12;
                           params: three 2^k x 2^k matrices (as DENSE),
                           U_1, U_2, U_3, where U_v acts on the targets
                           where bit(c_0) + 2 bit(c_1) = v; identity
                           where both are 0.  fuse() makes it from two
                           controlled dense gates on the same targets
                           (U_1, U_2 and their product)                   */
    SV_GATE_MUX3 = 14   /* as MUX2 with three controls (c_0, c_1, c_2) and
                           seven matrices U_1..U_7, v = bit(c_0) +
                           2 bit(c_1) + 4 bit(c_2); fuse() makes it from
                           three controlled dense gates                   */
} sv_gate_kind;

typedef struct sv_state sv_state;      /* device state vector + stream   */
typedef struct sv_circuit sv_circuit;  /* host gate list (+ device copy) */
typedef struct svb svb;                /* batch of small HHL solves      */
typedef struct svs svs;                /* serving loop                   */

/* Parameters of an HHL circuit (Sec. III-A step 1, Sec. III-B). */
typedef struct {
    int n_sys;        /* ns: system qubits, 2^ns >= dim                     */
    int n_clock;      /* m: clock (phase-estimation) qubits                 */
    int n_total;      /* ns + m + 1                                         */
    int n_qpe_est;    /* Sec. III-B estimate for the clock register         */
    int n_gates;      /* gates in the circuit                               */
    int dim;          /* N: rows of the caller's A                          */
    int j0;           /* clock value that stands for lambda_lo              */
    double t;         /* evolution time of e^{iAt}                          */
    double C;         /* inversion constant: ancilla |1> amplitude C/lambda  */
    double lambda_lo, lambda_hi, kappa;  /* over the eigenvectors b reaches */
    double b_norm;    /* ||b|| (step 1)                                     */
    int x_offset;     /* x is read at system indices x_offset .. + dim - 1 */
    int sign_qubit;   /* 1: the clock holds a two's-complement value       */
    int dilated;      /* 1: the circuit solves [[0, A'], [A'^T, 0]]        */
    int preconditioned; /* 1: Gauss-Seidel, the circuit solves M^{-1}A    */
} sv_hhl_info;

/* Result of postselection (Sec. III-A steps 3-4). */
typedef struct {
    double scale;          /* x = scale * x_hat = b_norm * ||Re y|| / C     */
    double p_anc1;         /* P(ancilla = 1)                                */
    double p_anc1_clock0;  /* P(ancilla = 1, clock = 0) = ||y||^2           */
    double max_imag;       /* max |Im y_s|                                  */
    double pad_leak;       /* ||y_s|| over padded indices s >= N            */
} sv_solution_info;

/* ---- states ----------------------------------------------------------- */

/* Allocate an n-qubit state (1 <= n <= 34) in device memory, initialised to
 * |0...0>, with its own stream.  SV_ERR_OOM if HBM is short. */
sv_status sv_create(int n_qubits, sv_dtype dtype, sv_state **out);

/* Wrap caller-owned device memory (e.g. a torch tensor) of at least
 * 2^n * amplitude-size bytes; the contents are left as they are.  The
 * memory must outlive the state.  The library links the system HIP runtime;
 * a torch build that bundles its own runtime must initialise it (first
 * torch.cuda call) before the library's first device call in the process. */
sv_status sv_create_from_buffer(void *dev_ptr, size_t bytes, int n_qubits,
                                sv_dtype dtype, sv_state **out);

/* Order the state's device work on a caller stream (hipStream_t, e.g.
 * torch.cuda.current_stream().cuda_stream); NULL restores the state's own. */
sv_status sv_set_stream(sv_state *s, void *hip_stream);

/* The state's device memory and stream, for callers that work on the
 * amplitudes themselves: *dev_ptr the device address of the 2^n amplitudes,
 * *bytes (may be NULL) their size, *hip_stream (may be NULL) the stream its
 * work is ordered on.  The state keeps ownership; the address is valid until
 * sv_destroy.  Host only. */
sv_status sv_device_buffer(const sv_state *s, void **dev_ptr, size_t *bytes,
                           void **hip_stream);

/* Free the state (and its memory unless adopted). */
sv_status sv_destroy(sv_state *s);

/* Reset to |0...0> (asynchronous). */
sv_status sv_reset(sv_state *s);

/* Copy count amplitudes starting at offset to/from host memory, in the
 * state's dtype (interleaved).  Synchronises the stream. */
sv_status sv_get_amplitudes(const sv_state *s, size_t offset, size_t count,
                            void *host_out);
sv_status sv_set_amplitudes(sv_state *s, size_t offset, size_t count,
                            const void *host_in);

/* Gather amplitudes at arbitrary indices (each < 2^n) into host_out
 * (count amplitudes, state dtype).  Synchronises the stream. */
sv_status sv_get_amplitudes_at(const sv_state *s, const uint64_t *indices,
                               size_t count, void *host_out);

/* sum |psi_i|^2, accumulated in double with a fixed reduction order.
 * Synchronises the stream. */
sv_status sv_norm2(const sv_state *s, double *out);

/* ---- circuits --------------------------------------------------------- */

/* Build the HHL circuit of Fig. 5 for A x = b (Sec. III-A):
 *   A: dim*dim row-major doubles, symmetric (|A - A^T| <= 1e-12 max|A|),
 *      positive definite on the span b reaches; b: dim doubles, nonzero.
 *   clock_bits: m in [1, 16]; t > 0 fixes the evolution time, t <= 0
 *   selects the rule that puts lambda_lo on clock value
 *   j0 = floor((2^m - 1) / kappa) (or lambda_hi on 2^m - 1 when kappa >
 *   2^m - 1).
 * The circuit: |b> preparation (a tree of uniformly controlled RY), H on the
 * clock, e^{iAt 2^j} controlled by clock bit j, inverse QFT, controlled-RY
 * inversion with angle 2 asin(min(1, j0 / c)) for clock value c >= 1, QFT,
 * the inverse controlled evolutions, H on the clock.
 * Errors: SV_ERR_NOT_SYMMETRIC, SV_ERR_NOT_POSDEF, SV_ERR_INVALID (b = 0,
 * dim < 1, m out of range, n > 34). */
sv_status circuit_build_hhl(const double *A, const double *b, int dim,
                            int clock_bits, double t, sv_circuit **out);

/* Flags for circuit_build_hhl_ex. */
enum {
    /* Keep the eigen-decomposition in the circuit and build the controlled
     * e^{iAt 2^j} matrices on the device (FP64) when the circuit is first
     * applied or added to a batch, instead of on the host at build time.
     * Host consumers that need them (circuit_serialize, fuse when the gate
     * fits in k_max) build them on demand. */
    SV_HHL_DEVICE_EVOLUTIONS = 1,
    /* Sign qubit (the n_neg qubit of Sec. III-B) for a symmetric A with
     * eigenvalues of either sign: the m clock qubits hold the eigenvalue
     * estimate in two's complement (-2^{m-1} .. 2^{m-1} - 1, m >= 2), the
     * automatic t maps max|lambda| to at most 2^{m-1} - 1, and the
     * inversion angle for decoded value v != 0 is 2 asin(clamp(j0 / v)),
     * negative for v < 0.  lambda_lo / lambda_hi / kappa are over |lambda|.
     * SV_ERR_SINGULAR when b reaches a zero eigenvalue. */
    SV_HHL_SIGNED = 2,
    /* Hermitian dilation (Sec. III-A step 1c) for a general square A: A is
     * padded to A' = A (+) I of size 2^k >= dim (step 1b), then the circuit
     * solves [[0, A'], [A'^T, 0]] [0; x] = [b; 0] on k + 1 system qubits
     * with the sign qubit (implies SV_HHL_SIGNED), and postselection reads
     * x from the second half (x_offset = 2^k).  dim <= 2048. */
    SV_HHL_DILATE = 4,
    /* Choose per input: SV_HHL_DILATE when A is not symmetric, else
     * SV_HHL_SIGNED when an eigenvalue b reaches is <= 0, else neither. */
    SV_HHL_AUTO = 8,
    /* Gauss-Seidel preconditioning (Sec. III-A step 1a, Sec. III-B): with
     * M = D + L, the lower triangle of A including the diagonal, the circuit
     * solves (M^{-1} A) x = M^{-1} b, which has the same solution and
     * usually a lower condition number.  M^{-1} A is not symmetric, so this
     * implies SV_HHL_DILATE; lambda_lo / lambda_hi / kappa / b_norm describe
     * the preconditioned system.  SV_ERR_SINGULAR on a zero diagonal entry. */
    SV_HHL_GAUSS_SEIDEL = 16
};

/* circuit_build_hhl with flags (0 = circuit_build_hhl). */
sv_status circuit_build_hhl_ex(const double *A, const double *b, int dim,
                               int clock_bits, double t, int flags,
                               sv_circuit **out);

/* Empty generic circuit on n qubits (1 <= n <= 34). */
sv_status circuit_create(int n_qubits, sv_circuit **out);

/* Append one gate (see sv_gate_kind for qubits and params).  Qubits must be
 * distinct and < n; nparams counts doubles. */
sv_status circuit_add_gate(sv_circuit *c, int kind, const int *qubits, int nq,
                           const double *params, int nparams);

/* HHL parameters (HHL circuits only; generic circuits fill n_total,
 * n_gates and zeros). */
sv_status circuit_info(const sv_circuit *c, sv_hhl_info *out);

/* Number of qubits and gates of any circuit. */
sv_status circuit_shape(const sv_circuit *c, int *n_qubits, int *n_gates);

/* Serialise the gate list.  With buf == NULL, *len receives the size.
 * Format (little-endian): int32 n_qubits, int32 n_gates, then per gate:
 * int32 kind, int32 nq, int32 nparams, nq int32 qubits, nparams float64. */
sv_status circuit_serialize(const sv_circuit *c, void *buf, size_t *len);

/* Gate fusion (Sec. II-C, Fig. 4): merge gates whose joint qubit set has at
 * most k_max (1..5) qubits into single DENSE (or DIAG when every member is
 * diagonal) gates.  Gates wider than k_max (controlled evolutions,
 * inversion) stay as they are.  The result is a new circuit with the same
 * unitary; products are formed in double precision. */
sv_status fuse(const sv_circuit *in, int k_max, sv_circuit **out);

/* Apply every gate of c to s, in order, asynchronously on s's stream.
 * SV_ERR_SHAPE if the circuit's qubit count differs from the state's. */
sv_status sv_apply(sv_state *s, const sv_circuit *c);

/* Kernel families reported by sv_apply_timed. */
typedef enum {
    SV_KERNEL_DENSE_DIRECT = 0, /* dense k <= 5, no target inside a 128-byte
                                   line (all >= 3 at c128, >= 4 at c64; at
                                   c64 also bit 0 alone inside the line):
                                   groups held in registers              */
    SV_KERNEL_DENSE_LDS = 1,    /* dense k <= 5, some target inside a line
                                   (at c128: three or more, or k = 5):
                                   LDS regroup                           */
    SV_KERNEL_DENSE_SMALL = 2,  /* dense k <= 5 on a state of < 6 + k qubits   */
    SV_KERNEL_DIAG = 3,         /* diagonal gate                                */
    SV_KERNEL_WIDE = 4,         /* dense gate on 6..12 targets, optional control */
    SV_KERNEL_UCRY = 5,         /* uniformly controlled RY                      */
    SV_KERNEL_DENSE_BFLY = 6,   /* dense k <= 4 at c128 with one or two targets
                                   inside a line: cross-lane butterfly, groups
                                   held in registers                     */
    SV_KERNEL_DENSE_MFMA = 7    /* dense k = 5 on >= 9 qubits, or k = 4 with
                                   two targets inside a line (at c64: one
                                   or two) on >= 8; every target inside a
                                   line among the two lowest: 16x16x4
                                   matrix-core products                  */
} sv_kernel_family;

/* As sv_apply, and record the device time of each gate's launch with HIP
 * events on the state's stream: launch_ms[g] for gate g (cap >= n_gates);
 * kernel_ids (may be NULL) receives each launch's sv_kernel_family.
 * Synchronises the stream. */
sv_status sv_apply_timed(sv_state *s, const sv_circuit *c, double *launch_ms,
                         int *kernel_ids, int cap);

/* Wait for all work queued on the state's stream. */
sv_status sv_synchronize(sv_state *s);

/* Postselection and recovery (Sec. III-A steps 3-4): y_s = psi[2^{n-1} + s]
 * (ancilla 1, clock 0); x_hat = Re(y)/||Re y|| over the first dim entries;
 * info->scale = b_norm * ||Re y|| / C so that x = scale * x_hat.  Sums are
 * accumulated in double.  dim must equal the circuit's.  Synchronises. */
sv_status sv_postselect_solution(sv_state *s, const sv_circuit *hhl,
                                 double *x_hat, int dim,
                                 sv_solution_info *info);

/* Step 4b of Sec. III-A: x = info->scale * x_hat, elementwise over dim
 * entries, into the caller's x (dim doubles).  SV_ERR_INVALID on a NULL
 * pointer or dim < 1.  Host only. */
sv_status sv_solution_x(const double *x_hat, int dim,
                        const sv_solution_info *info, double *x);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * readout of sv_postselect_solution, with the same results, on a state the
 * caller owns.  dev_psi: device pointer to the 2^n_qubits amplitudes of
 * dtype (bytes = its size, at least 2^n_qubits amplitudes); hip_stream: the
 * stream the work is ordered on (NULL = the null stream); hhl, x_hat, dim
 * and info as in sv_postselect_solution.  Allocates nothing: the reduction
 * partials and the postselected block go to a fixed device array of
 * 1024 + 2 + 2*1024 doubles per GPU (about 24 KiB, held until the process
 * ends), so the circuit may have at most 10 system qubits (SV_ERR_SHAPE
 * beyond).  Calls that overlap on one GPU share that array and race.
 * Synchronises hip_stream. */
sv_status sv_postselect_solution_noalloc(const void *dev_psi, size_t bytes,
                                         int n_qubits, sv_dtype dtype,
                                         void *hip_stream,
                                         const sv_circuit *hhl,
                                         double *x_hat, int dim,
                                         sv_solution_info *info);

sv_status circuit_destroy(sv_circuit *c);

/* ---- batched solves --------------------------------------------------- */
/* Many small HHL solves in persistent launches, captured once in a hipGraph
 * and replayed by later svb_run calls.  Instances whose state fits in 64 KiB
 * (n <= 12 at complex128, n <= 13 at complex64) run one workgroup per state
 * with the state in LDS, one launch per size class; larger ones run through
 * the whole-GPU sweep kernels in groups of up to 64 same-shape instances
 * (one launch per fused op for the group).  Every instance's arithmetic is
 * independent of the rest of the batch.
 *
 * svb_create: k_max in 1..5 fuses every instance with that width; 0 uses the
 * width svb_autotune chose for the instance's (ns, m), else 3.  hip_stream may
 * be NULL (own stream).
 * svb_add: copies and fuses an HHL circuit (<= 24 qubits); *index_out gets
 * its index.  Adding invalidates the device copy (re-uploaded by svb_run).
 * svb_run: runs every instance; synchronises.  SV_ERR_OOM if HBM is short.
 * svb_solution: the instance's x_hat (unit norm, dim entries) and info as in
 * sv_postselect_solution.  svb_last_run_ms: device time of the last run
 * (HIP events around the graph launch). */
sv_status svb_create(sv_dtype dtype, int k_max, void *hip_stream, svb **out);
sv_status svb_add(svb *bt, const sv_circuit *hhl, int *index_out);
sv_status svb_run(svb *bt);
sv_status svb_solution(svb *bt, int index, double *x_hat, int dim,
                       sv_solution_info *info);
/* svb_postselected: the raw postselected block of instance `index` (Sec.
 * III-A step 3): y_s = psi[2^{n-1} + s] for s < count (count <= 2^ns), as
 * 2*count doubles (re, im) widened from the instance's dtype, and
 * P(ancilla = 1) into *p_anc1 (may be NULL).  SV_ERR_INVALID before the
 * first svb_run or for a bad index, SV_ERR_SHAPE if count > 2^ns. */
sv_status svb_postselected(svb *bt, int index, double *y, int count,
                           double *p_anc1);
sv_status svb_last_run_ms(const svb *bt, double *ms);
/* svb_run_timed: the launches of svb_run without its graph, one work item
 * after another on the batch's stream, each timed with HIP events, for a
 * breakdown of the batch's device time.  An item is a size class of the
 * batched kernel (kind 0) or a group of same-shape instances run through the
 * whole-GPU sweep kernels (kind 1).  For item i < *items: n[i] qubits,
 * count[i] instances, ops[i] fused ops per instance (the most in a class),
 * ms[i] device time.  The arrays hold cap entries; SV_ERR_INVALID (with
 * *items set) if cap is below the number of items.  Leaves the results as
 * svb_run does; svb_last_run_ms then gives the sum of the items. */
sv_status svb_run_timed(svb *bt, int cap, int *items, int *kind, int *n,
                        int *count, int *ops, double *ms);
/* svb_run_timed_ops: as svb_run_timed for the grouped sweeps only, with each
 * fused op's launch timed on its own (HIP events on the batch's stream), for
 * a breakdown of the sweeps by kernel family.  For entry i < *count (one per
 * op of every group, groups in svb_run_timed's item order): item[i] the
 * group's item index in svb_run_timed, family[i] the sv_kernel_family used,
 * k[i] the op's targets (UCRY: controls), controlled[i] the control qubits
 * of a wide gate (0, 1, or 2 for a MUX2 gate), ms[i] device time.  Arrays hold cap entries;
 * SV_ERR_INVALID (with *count set) if cap is too small.  The outputs it
 * leaves are not a run's results: call svb_run afterwards. */
sv_status svb_run_timed_ops(svb *bt, int cap, int *count, int *item, int *family,
                            int *k, int *controlled, double *ms);
sv_status svb_size(const svb *bt, int *count);
sv_status svb_destroy(svb *bt);

/* ---- serving ----------------------------------------------------------- */
/* Continuous-batching server for HHL solves on one GPU.  svs_submit copies
 * the inputs and queues the request; prep threads build each circuit (the
 * controlled evolutions are built on the device), fuse it, wait until its
 * device footprint fits in the HBM budget and a slot is free (admission),
 * and upload it.  A scheduler keeps several micro-batches in flight on
 * separate streams: requests whose state fits in LDS run together in the
 * batched persistent kernel (optionally also larger ones with their state in
 * HBM); the others run through the sweep kernels, launched by a few launcher
 * threads with a stream each, and requests of the same shape waiting
 * together share launches (each fused op applied to every member's state,
 * with that member's own matrices, in one launch).
 * Requests that arrive while others are on the GPU are admitted as memory
 * and slots free up.  A request's result does not depend on what else is
 * in flight.  All svs_* calls are thread-safe.
 *
 * svs_start: hbm_budget_bytes = 0 uses half of the free HBM; max_slots
 *   bounds the requests resident at once.
 * svs_configure: before the first submit (SV_ERR_BUSY after).
 * svs_submit: dim in [1, 4096], clock_bits in [1, 16]; SV_ERR_BUSY when the
 *   queue limit is reached (counted as rejected).  *ticket identifies it.
 * svs_poll: SV_PENDING until done; then SV_OK with x_hat (dim entries,
 *   unit norm) and info as in sv_postselect_solution, or the request's
 *   error (SV_ERR_OOM when it can never fit the budget or its allocation
 *   failed, SV_ERR_NOT_SYMMETRIC / SV_ERR_NOT_POSDEF / SV_ERR_INVALID from
 *   the build, SV_ERR_INVALID if cancelled).  A finished ticket is consumed
 *   by the poll that returns it.
 * svs_cancel: cancels a request that has not been admitted yet.
 * svs_drain: waits until every submitted request has finished (timeout_s
 *   <= 0: no limit; SV_ERR_BUSY on timeout).
 * svs_stats: latency = finish - submit (host monotonic clock); p50 / p99 by
 *   nearest rank over the exact sorted sample of successful requests;
 *   solves/s = successful requests / (last finish - first submit).
 * svs_stop: drains, joins the threads and frees the server. */
enum {
    SVS_OPT_PREP_THREADS = 1,  /* host build threads (default min(8, cores/2)) */
    SVS_OPT_K_MAX = 2,         /* fusion width (0: the tuned width for batched
                                  shapes; for the others 3 below 18 qubits,
                                  5 from 18; default 0)                       */
    SVS_OPT_MAX_BATCH = 3,     /* requests per batched launch (default 256)      */
    SVS_OPT_STREAMS = 4,       /* micro-batches in flight (default 8)            */
    SVS_OPT_QUEUE_LIMIT = 5,   /* queued, not yet admitted requests              */
    SVS_OPT_FAIL_ALLOC_AT = 6, /* failure injection: the n-th request device
                                  allocation fails as out of memory (0 = off)  */
    SVS_OPT_BATCH_MAX_QUBITS = 7, /* also batch requests of up to this many
                                  qubits with the state in HBM (default 0:
                                  none)                                       */
    SVS_OPT_HHL_FLAGS = 8,     /* SV_HHL_SIGNED | _DILATE | _AUTO |
                                  _GAUSS_SEIDEL for every request's circuit
                                  (default 0)                                 */
    SVS_OPT_LAUNCHERS = 9,     /* threads (each with its own stream) that
                                  launch the requests not batched (default 4) */
    SVS_OPT_GROUP_WINDOW_US = 10, /* microseconds a request not batched may
                                  wait for others of its shape to share its
                                  launches (default 0: launch at once)        */
    SVS_OPT_LDS_MAX_QUBITS = 11 /* batch a request with its state in LDS only
                                  up to this many qubits, if its state fits
                                  (-1: every state that fits, n <= 12 at
                                  complex128, n <= 13 at complex64; default 0:
                                  none, every request runs on the grouped
                                  whole-GPU sweeps, which gave the lower
                                  latency under load)                         */
};
sv_status svs_start(size_t hbm_budget_bytes, int max_slots, sv_dtype dtype,
                    svs **out);
sv_status svs_configure(svs *srv, int option, double value);
sv_status svs_submit(svs *srv, const double *A, const double *b, int dim,
                     int clock_bits, double t, uint64_t *ticket);
sv_status svs_poll(svs *srv, uint64_t ticket, double *x_hat, int dim,
                   sv_solution_info *info);
/* As svs_poll; when the request is done also copies its raw postselected
 * block y_s = psi[2^{n-1} + s], s < y_count (y_count <= 2^ns; y may be NULL)
 * as 2*y_count doubles (re, im), and P(ancilla = 1) into *p_anc1 (may be
 * NULL).  SV_ERR_SHAPE if y_count > 2^ns; the ticket is consumed as by
 * svs_poll. */
sv_status svs_poll_ex(svs *srv, uint64_t ticket, double *x_hat, int dim,
                      sv_solution_info *info, double *y, int y_count,
                      double *p_anc1);
sv_status svs_cancel(svs *srv, uint64_t ticket);
sv_status svs_drain(svs *srv, double timeout_s);
sv_status svs_stats(svs *srv, double *p50_s, double *p99_s,
                    double *solves_per_s, uint64_t *n_rejected);
sv_status svs_counts(svs *srv, uint64_t *done, uint64_t *failed,
                     uint64_t *pending);
/* Mean seconds per successful request in each phase: out[0] queue (submit
 * to prep start), out[1] build + fuse + admission wait, out[2] upload,
 * out[3] resident to launched, out[4] launched to results back; out[5] /
 * out[6] requests run batched / through the sweep kernels; out[7] prep
 * threads; with cap >= 10, out[8] / out[9] grouped launches of two or more
 * same-shape requests / the requests in them.  cap >= 8. */
sv_status svs_profile(svs *srv, double *out, int cap);
sv_status svs_stop(svs *srv);

/* Launch choices of batch instances of one shape (dtype, ns, m). */
typedef struct {
    int k_max;         /* fusion width, 1..5                                  */
    int group_max;     /* instances per grouped launch of states in HBM
                          (at most 256)                                        */
    int wave_target;   /* waves a grouped wide-gate launch aims to keep busy
                          when it picks rows per wave                          */
    int resident_kib;  /* largest state, in KiB, run with the state in LDS
                          (a power of two up to 128; default 64); larger
                          ones run as grouped sweeps                          */
    int tuned;         /* 1: chosen by the autotuner, 0: the defaults         */
    double ms;         /* device time of the choice on the tuning batch       */
} svb_tune;

/* Autotuner: time batches of `copies` copies of `sample` (for a batch, the
 * number of its instances of that shape is representative) and record the
 * fastest launch choices for the sample's (dtype, ns, m), used by batches
 * created with k_max = 0.  Coordinate descent from the defaults (k 3, groups
 * of 256, wave target 1024, LDS residency up to 64 KiB): k_max = 1..5 first
 * (device times into ms_per_k, 5 entries, may be NULL); then, for a state of
 * 64..128 KiB, residency in LDS, and for one of 16..64 KiB, the grouped
 * sweeps instead (at the tuned k and one wider); then, for a state that runs
 * as grouped sweeps, groups of 64 and wave targets of 256 and 4096.  A trial's time is
 * the sum of its launches run one work item after another (svb_run_timed),
 * the cost the shape adds to a large batch.  k_max and
 * residency change the arithmetic order (the results stay within the parity
 * bars); the other choices do not.  *out (may be NULL) gets the choice. */
sv_status svb_autotune_ex(sv_dtype dtype, const sv_circuit *sample, int copies,
                          svb_tune *out, double *ms_per_k);
/* As svb_autotune_ex; returns the chosen k_max only. */
sv_status svb_autotune(sv_dtype dtype, const sv_circuit *sample, int copies,
                       int *best_k, double *ms_per_k);
/* The recorded choices for a shape (the defaults, tuned = 0, if none). */
sv_status svb_get_tune(sv_dtype dtype, int ns, int m, svb_tune *out);
/* Record choices for a shape (e.g. a saved tuning table), as the autotuner
 * would; t->tuned and t->ms are ignored.  SV_ERR_INVALID outside k_max 1..5,
 * group_max 1..256, wave_target >= 1, resident_kib a power of two up to
 * 128. */
sv_status svb_set_tune(sv_dtype dtype, int ns, int m, const svb_tune *t);

const char *sv_last_error(void);

/* Test hook: bound the workgroups of every kernel launch made after the call
 * by max_workgroups (0 = no bound, the default).  Every kernel walks its
 * tiles or rows with a grid-wide (or per-XCD) loop, so the bound changes
 * which wave takes which tile, not the arithmetic of any output element; it
 * lets small states drive the multi-tile loops that large states take.
 * Graphs captured earlier keep their launch shapes.  Process-wide; not for
 * use while other threads launch.  SV_ERR_INVALID if negative. */
sv_status sv_debug_set_grid_cap(int max_workgroups);

/* Achievable-bandwidth probe: reps launches, each reading every amplitude of
 * a complex128 state of >= 10 qubits and writing it back unchanged, with the
 * access shape, grid and per-XCD tile slices of the dense sweep kernels;
 * launch_ms[r] (reps entries) receives each launch's device time (HIP
 * events on the state's stream).  Algorithmic bytes per launch: 2 * 16 *
 * 2^n.  The state is unchanged.  Synchronises.  SV_ERR_SHAPE for another
 * dtype or fewer qubits. */
sv_status sv_stream_probe(sv_state *s, int reps, double *launch_ms);

/* Select the form of 5-qubit dense gates, and of 4-qubit gates with targets
 * inside a cache line, for launches made after the call: enable = 1
 * (the default) the matrix-core kernel where it applies, 0 the vector
 * kernels everywhere, 2 the matrix-core kernel also for every other 4-qubit
 * gate it can take (no third target inside a line).  SV_ERR_INVALID for
 * other values.  Both compute the same gate (Sec. II-C fused
 * gates); the switch exists to compare and test them.  Process-wide; not for
 * use while other threads launch; graphs captured earlier keep their
 * kernels. */
sv_status sv_debug_set_dense_mfma(int enable);

/* Select the kernel of complex64 dense gates whose only target inside a
 * 128-byte line is bit 0, for launches made after the call: enable != 0 (the
 * default) the register kernel that moves amplitude pairs (a pair holds two
 * entries of one group), 0 the LDS regroup.  Same gate either way; for
 * comparison and tests.  Process-wide, as sv_debug_set_dense_mfma. */
sv_status sv_debug_set_pair0(int enable);

/* Sec. III-B qubit estimate, in the reading that reproduces Table I:
 * n_data = ceil(log2 dim), n_qpe = max(n_data + 1, ceil(log2(kappa + 1)))
 * + has_negative, n_total = n_data + n_qpe + 1 (inversion ancilla). */
sv_status sv_qubit_estimate(int dim, double kappa, int has_negative,
                            int *n_data, int *n_qpe, int *n_total);

/* ---- Newton-Raphson AC power flow ------------------------------------- */
/* The power-flow use case of Sec. III: Newton-Raphson on the polar AC
 * power-flow equations with HHL as the linear solver of every iteration.
 *
 * Case (all arrays caller-owned, read only): buses 0..n_bus-1 with
 * bus_type 0 (slack, exactly one), 1 (PV) or 2 (PQ); branch e joins from[e]
 * and to[e] with series impedance r[e] + j x[e] and total line charging
 * b_charging[e] (per unit); p_spec / q_spec: net injected power (generation
 * minus load); v_set: the voltage magnitude held at slack and PV buses.
 * Unknowns: the angles of the non-slack buses, then the magnitudes of the
 * PQ buses, in bus order (n_unknowns of them).
 *
 * pf_mismatch_jacobian (host only): at magnitudes vm and angles va (n_bus
 * each), the injections P, Q (n_bus), the mismatch F = [p_spec - P;
 * q_spec - Q] over the unknowns' buses (n_unknowns) and the Jacobian
 * d[P; Q]/d[angles; magnitudes] (n_unknowns^2, row-major); any output may be
 * NULL.  SV_ERR_INVALID on a malformed case.
 *
 * pf_newton_hhl: flat start, then for at most max_iter iterations builds the
 * HHL circuit of J dx = F (circuit_build_hhl_ex with clock_bits, automatic t
 * and hhl_flags: SV_HHL_DILATE, SV_HHL_GAUSS_SEIDEL or SV_HHL_AUTO, plus
 * optionally SV_HHL_DEVICE_EVOLUTIONS; with none of the first three,
 * SV_HHL_DILATE), fuses it to k_max (0: unfused), runs it on the GPU at
 * dtype, takes dx = info.scale * x_hat from sv_postselect_solution and
 * updates; stops when max |F| < tol.  vm, va (n_bus) receive the operating
 * point; *info (may be NULL) the iteration record.  Errors from the HHL
 * calls are returned as they are. */
#define PF_HISTORY 64
typedef struct {
    int iterations;     /* updates applied                                */
    int converged;      /* max |F| < tol reached                           */
    int n_unknowns;
    double mismatch;    /* final max |F|                                   */
    double hhl_seconds; /* host wall time spent in the HHL solves          */
    double history[PF_HISTORY];   /* max |F| before each update            */
} pf_info;

sv_status pf_mismatch_jacobian(int n_bus, int n_branch, const int *from,
                               const int *to, const double *r,
                               const double *x, const double *b_charging,
                               const int *bus_type, const double *p_spec,
                               const double *q_spec, const double *vm,
                               const double *va, double *P, double *Q,
                               double *F, double *J, int *n_unknowns);
sv_status pf_newton_hhl(int n_bus, int n_branch, const int *from,
                        const int *to, const double *r, const double *x,
                        const double *b_charging, const int *bus_type,
                        const double *p_spec, const double *q_spec,
                        const double *v_set, int clock_bits, int hhl_flags,
                        sv_dtype dtype, int k_max, int max_iter, double tol,
                        double *vm, double *va, pf_info *info);

#ifdef __cplusplus
}
#endif
#endif
