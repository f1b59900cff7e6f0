/*
 * qcw.h -- C ABI of the MI355X (gfx950) gate-sweep library.
 *
 * The library applies QCWAVE's k-qubit operators (Tabakin & Julia-Diaz,
 * "QCWAVE - a Mathematica quantum computer simulation update",
 * arXiv:1101.1785) to complex FP64 state vectors held in GPU memory.
 *
 * Conventions shared by every call (paper §2c Eq. staten; §3a-§3c):
 *   - A state of nq qubits is 2^nq amplitudes of qcw_c64 (16 bytes, re then
 *     im), contiguous, amplitude C_n at offset n, where
 *     n = sum_i q_i 2^(nq-i).  Qubit 1 is the MOST significant bit of n, so
 *     qubit `is` owns bit nq - is and has stride 2^(nq-is).
 *   - Qubits are numbered 1..nq, as in the paper's Op1/Op2/Op3 calls.
 *   - A k-qubit gate (k = 1, 2, 3) is an m x m complex matrix, m = 2^k,
 *     row-major, U[r*m + c] = <r|U|c>.  The local index r lists the values
 *     of the targets in ARGUMENT order, the first target most significant:
 *     r = sum_j q_{is_j} 2^(k-j).  For k = 2 this is V_{ij;kl} = <ij|V|kl>
 *     with i the value of is1 (§3b, Eq. resmat2); k = 3 extends it the same
 *     way (§3c omits the derivation).  Any order of distinct targets is
 *     allowed: CNOT with control 3 and target 1 is qcw_op2(CNOT, 3, 1, ...).
 *   - Matrices need not be unitary: the sweep is linear in U, and noise or
 *     Kraus operators are scaled unitaries.  States are never renormalised.
 *
 * Memory and ownership:
 *   - `psi`, `psi_in`, `psi_out` are DEVICE pointers owned by the caller;
 *     each must lie inside one device allocation that holds all 2^nq
 *     amplitudes (checked; a buffer that is too short is rejected).
 *   - Gate matrices, gate lists and target arrays are HOST pointers; they
 *     are consumed before the call returns and may be freed right after.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously on it; the call does not synchronise unless its
 *     description says so (the fused passes and OmegaALL when they upload a
 *     new pass plan, the observables, eigenvalue and autotune calls).
 *
 * Errors: every call returns QCW_OK or a negative code synchronously and
 * raises no exception.  QCW_EINVAL: null pointer, nq outside [1, 34],
 * k outside {1, 2, 3} or k > nq, a target outside [1, nq], repeated targets,
 * a pointer that is not device memory or a buffer shorter than the state,
 * or partially overlapping input and output.  QCW_EHIP: a HIP runtime call
 * or kernel launch failed.  Faults inside kernels surface at the caller's
 * next synchronisation of the stream.  qcw_last_error() returns a
 * thread-local description of the most recent failure.
 *
 * Threading: calls on different streams may run from different threads.
 */
#ifndef QCW_H
#define QCW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} qcw_c64; /* same layout as complex128 / hipDoubleComplex */

enum {
  QCW_OK = 0,
  QCW_EINVAL = -1,
  QCW_ENOMEM = -2,
  QCW_EHIP = -3,
  QCW_EAGAIN = -4
};

/* Human-readable name of an error code (static string). */
const char *qcw_strerror(int code);
/* Description of the calling thread's most recent failure ("" if none). */
const char *qcw_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int qcw_version(void);

/*
 * Op1 (§3a, Eqs. oneopres and resmat1): for each of the 2^nq / 2 partner
 * pairs (n0, n1 = n0 + 2^(nq-is)), (C_n0, C_n1) <- U (C_n0, C_n1), in place.
 * U: host, 2 x 2.  The paper's psi_f = Op1[U, is, psi_0].
 */
int qcw_op1(const qcw_c64 *U, int is, qcw_c64 *psi, int nq, void *stream);

/*
 * Op2 (§3b, Eqs. twoopA and resmat2): for each of the 2^nq / 4 amplitude
 * quartets (n00, n01, n10, n11), with n01 = n00 + 2^(nq-is2) and
 * n10 = n00 + 2^(nq-is1), the quartet is multiplied by the 4 x 4 V, in place.
 */
int qcw_op2(const qcw_c64 *V, int is1, int is2, qcw_c64 *psi, int nq,
            void *stream);

/*
 * Op3 (§3c and §4c): the 8 x 8 W on each of the 2^nq / 8 amplitude octets of
 * qubits is1, is2, is3 (local index 4 q_is1 + 2 q_is2 + q_is3), in place.
 */
int qcw_op3(const qcw_c64 *W, int is1, int is2, int is3, qcw_c64 *psi, int nq,
            void *stream);

/* Op_k for k = 1, 2, 3 with targets[0..k-1]; in place. */
int qcw_opk(int k, const int *targets, const qcw_c64 *U, qcw_c64 *psi, int nq,
            void *stream);

/*
 * Functional form psi_out = Op_k(psi_in), as the paper's commands return a
 * new state (§3a footnote).  psi_in == psi_out is allowed (in place); any
 * other overlap of the two buffers is rejected.
 */
int qcw_opk_to(int k, const int *targets, const qcw_c64 *U,
               const qcw_c64 *psi_in, qcw_c64 *psi_out, int nq, void *stream);

/* OmegaALL[U, psi] (§4a): the same 2 x 2 U on every qubit, qubit 1 first.
 * From 22 qubits on it runs as list-order fused passes (about nq/8 passes
 * over HBM instead of nq sweeps; bit for bit the same result, and the stream
 * is synchronised once when the pass plan changes, as in qcw_circuit_fused). */
int qcw_omega_all(const qcw_c64 *U, qcw_c64 *psi, int nq, void *stream);

/*
 * A gate of a circuit: k targets q[0..k-1] (1-based; unused entries
 * ignored) and the offset, in qcw_c64 elements, of its m x m matrix inside
 * the circuit's `mats` array.
 */
typedef struct {
  int32_t k;
  int32_t q[3];
  int64_t mat;
} qcw_gate;

/*
 * A circuit: the gates applied in list order, i.e. the operator product read
 * right to left (CNOT_12 H_1 |00> applies H_1 first; §5).  Plain form: one
 * sweep per gate on `stream`; on states of at most 11 qubits the gates run in
 * one launch (a further launch per 32 gates or 224 matrix entries) with the
 * state in LDS, each gate the sweep's group update, bit for bit one sweep per
 * gate.  gates, mats: host arrays, read before the call returns; nmats is the
 * length of mats in qcw_c64 elements (every gate's matrix must lie inside it).
 */
int qcw_circuit(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                const qcw_c64 *mats, int64_t nmats, void *stream);

/*
 * The same circuit with the same result, bit for bit, in fewer passes over
 * HBM: consecutive gates whose targets fit, together with the lowest label
 * bits (4 by default: 256-byte chunks), in `tile_bits` bits (8..13; 0 = the tuned default, 12) form one pass.  A pass loads each
 * tile of 2^tile_bits amplitudes (fixed values of the other bits) into LDS,
 * applies every gate of the run there with the one-gate sweep's arithmetic,
 * and stores it back, so a run of gates costs one read and one write of the
 * state instead of one per gate.  States below 9 qubits use one sweep per
 * gate.  Synchronises `stream` once, to hand the pass plan to the device,
 * unless the stream's previous call had the same request (shape, flags,
 * gates and matrix entries): its plan is kept on the device per stream and
 * reused, and the call then only enqueues the passes.
 */
int qcw_circuit_fused(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                      const qcw_c64 *mats, int64_t nmats, int tile_bits, void *stream);
/* Plan flags for qcw_circuit_fused_ex (0: passes are runs of consecutive
 * gates and the result equals qcw_circuit bit for bit).  Each flag leaves the
 * circuit's operator unchanged and changes only the rounding: results equal
 * qcw_circuit to FP64 rounding. */
enum {
  /* A gate may join an earlier pass ahead of gates that were deferred to a
   * later one, provided it shares no qubit with any of them: gates on
   * disjoint qubits commute (the tensor structure of §2c), and gates sharing
   * a qubit keep their order.  A random 124-gate circuit on 31 qubits takes
   * 11 passes instead of 17. */
  QCW_PLAN_COMMUTE = 1,
  /* Inside each pass, consecutive gates spanning at most three qubits become
   * one gate (their product, computed on the host), so a tile goes through
   * LDS fewer times (124 gates become about 70 for the circuit above). */
  QCW_PLAN_FUSE = 2,
  /* Each gate inside a tile uses the three-product form of the complex
   * matrix-vector product (U = A + iB on x = a + ib: Re y = A(a+b) - (A+B)b,
   * Im y = A(a+b) + (B-A)a, with A+B and B-A formed on the host): 3m instead
   * of 4m FMAs per amplitude for an m x m gate.  Its rounding error stays
   * within a small factor of the direct product's for matrices of modest
   * norm, such as unitaries. */
  QCW_PLAN_3M = 4,
};

/* The same with the number of contiguous low label bits every tile keeps
 * (low_bits, 3..5; 0 = the tuned default): tiles are made of 2^low_bits-
 * amplitude contiguous chunks, and tile_bits - low_bits <= 10 bits are left for
 * the gates' targets; the threads per tile (256 or 512 for tile_bits 11;
 * 256, 512 or 1024 for 12 and 13, where 12 with 1024 is a warp-specialised
 * pipelined kernel; 0 = the tuned default); and the plan flags
 * (any of QCW_PLAN_COMMUTE | QCW_PLAN_FUSE | QCW_PLAN_3M, or 0; other bits are
 * QCW_EINVAL). */
int qcw_circuit_fused_ex(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                         const qcw_c64 *mats, int64_t nmats, int tile_bits, int low_bits,
                         int threads, int plan, void *stream);
/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): qcw_circuit_fused_ex
 * with the same arguments, kernels and results (bit for bit), except that the
 * pass and gate tables of the plan are kept in a static device array of the
 * library, 4 MiB on each GPU that the library runs on (held until the process
 * ends), instead of a buffer allocated per stream.  The call allocates no
 * device memory and frees none.  A plan whose tables exceed 4 MiB is rejected
 * with QCW_EINVAL (the benchmark's 124-gate plan at 31 qubits takes about
 * 0.16 MiB; each pass costs 8.3 KiB and each gate after in-pass fusion
 * 1.6 KiB).  All calls on one GPU share its array, which keeps the last plan:
 * the same request again reuses it without planning, upload or
 * synchronisation; a new request plans, uploads on `stream` and synchronises
 * it once.  Calls that overlap on one GPU (on different streams or threads,
 * with different requests) race on the array.
 */
int qcw_circuit_fused_noalloc(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                              const qcw_c64 *mats, int64_t nmats, int tile_bits, int low_bits,
                              int threads, int plan, void *stream);
/* Number of passes qcw_circuit_fused_ex makes for this gate list and plan
 * (host only; QCW_PLAN_FUSE and QCW_PLAN_3M do not change it). */
int qcw_fused_pass_count(int nq, const qcw_gate *gates, int ngates, int tile_bits,
                         int low_bits, int plan);
/* The same plan in full (host only): pass_of[g] receives the pass of gate g
 * (0-based), order[0..ngates) the gate indices in the order the passes apply
 * them (before any QCW_PLAN_FUSE merging).  pass_of and order are caller-owned
 * host arrays of ngates ints.  Returns the pass count, or a negative code.
 * States below 9 qubits (or tile_bits < 8) run one sweep per gate: pass_of[g]
 * = g and the list order. */
int qcw_fused_plan(int nq, const qcw_gate *gates, int ngates, int tile_bits, int low_bits,
                   int plan, int *pass_of, int *order);

/*
 * Test only (host code; no GPU is touched): the pass plan that
 * qcw_circuit_fused_ex would upload for this request (nq >= 9), as the device
 * tables hold it.  Pass p (p < *npass <= pass_cap): pass_hdr[4p .. 4p+3] =
 * {first gate in the gate table, gate count, tile bits T, low bits L};
 * outer_pos[40p + j] = the label bit of bit j of the block index (j < nq - T;
 * -1 beyond); chunk_off[1024p + c] = the label offset of chunk c of the tile
 * (c < 2^(T-L)).  The kernels give the amplitude of local index i (0 <= i <
 * 2^T) in the tile of block b the label
 *   sum_j bit_j(b) 2^outer_pos[j] + chunk_off[i >> L] + (i & (2^L - 1)).
 * Gate g (g < *ngate <= gate_cap): gate_hdr[13g .. 13g+12] = {k, sb0, sb1,
 * sb2 (local target bits, ascending), m3 (1: the three-product form), off[0..7]
 * (local member offsets, local index order)}; gate_mat[64g ...] its m x m
 * matrix row-major (with m3, the pairs (Re U, -(Re U + Im U))).  All arrays
 * are caller-owned host memory.  Returns QCW_OK or QCW_EINVAL (also when a cap
 * is too small; *npass and *ngate then hold the sizes needed).
 */
int qcw_debug_fused_tables(int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
                           int64_t nmats, int tile_bits, int low_bits, int plan, int pass_cap,
                           int gate_cap, int32_t *pass_hdr, int32_t *outer_pos,
                           uint64_t *chunk_off, int32_t *gate_hdr, qcw_c64 *gate_mat,
                           int *npass, int *ngate);

/*
 * One GPU's part of a gate on a state split over two GPUs by qubit 1 (the most
 * significant bit, §2c), the distribution of the paper's MPI predecessor (§5,
 * general remarks).  The full state has nq qubits (2 <= nq <= 34); this GPU's
 * share psi_local holds, in label order, the 2^(nq-1) amplitudes whose qubit
 * 1 equals rank_bit (0 or 1); psi_remote holds the partner's share as received
 * before this gate (read only; must not overlap psi_local).  Targets are in
 * the full state's numbering.  If qubit 1 is a target, psi_local becomes this
 * GPU's half of the gate applied to the whole state; run on both halves (each
 * with the other's pre-gate share as psi_remote) the result equals qcw_opk on
 * the whole state, bit for bit.  Otherwise the gate is the one-gate sweep on
 * the share and psi_remote is not read.  Device buffers, asynchronous on
 * stream; the exchange itself is the caller's.
 */
int qcw_op_shard(int k, const int *targets, const qcw_c64 *U, int rank_bit, qcw_c64 *psi_local,
                 const qcw_c64 *psi_remote, int nq, void *stream);

/*
 * Pick_k as computed by the device (§4a-§4c): writes (2^nq / m) * m labels to
 * the HOST array out_host, group after group in ascending base label, the
 * members of a group in ascending local index.  nq <= 26.  Synchronous.
 * For testing the device's index arithmetic.
 */
int qcw_debug_pick_device(int nq, int k, const int *targets, uint64_t *out_host);

/*
 * Batched form: many independent (state, circuit) instances -- the paper's
 * independent multiverse paths, each evolved by its own gate sequence (§5,
 * "The multiverse approach") -- advanced in ONE persistent launch.
 *
 * Instance i has nq qubits, its state at states + state_off (2^nq qcw_c64,
 * in the device buffer `states` of nstates elements, caller-owned) and its
 * circuit gates[gate_off .. gate_off + ngates - 1] (host array of ngates_total
 * entries; each gate's matrix at mats + gate.mat, host array of nmats).
 * Instances of up to 11 qubits keep their state in one wavefront's LDS for the
 * whole circuit; larger ones run as plain sweeps in the same graph.  Instance
 * states must not overlap.  A gate row may be shared by instances of equal nq.
 *
 * qcw_batch_create validates everything, copies gates and matrices to the
 * device, chooses each instance's tile shape from `tune_table` (a file written
 * by qcw_batch_autotune; NULL = built-in defaults; a table written for another
 * GPU architecture is rejected), and captures the launch in a hipGraph on
 * `stream` (NULL: a private stream).  qcw_batch_run replays the graph on
 * `stream`: every instance's state advances by its whole circuit, in place.
 * The handle owns its device copies and the graph; qcw_batch_destroy frees
 * them (never the caller's states).  With the exact tile shapes (every shape
 * but "amp4_mfma") results equal, bit for bit, those of qcw_circuit applied
 * to each instance alone.  "amp4_mfma" fuses each circuit (qcw_fuse_circuit,
 * at most three qubits per gate) and applies two- and three-qubit gates with
 * FP64 matrix-core instructions: results then agree with qcw_circuit to FP64
 * rounding, and still do not depend on the other instances of the launch.
 */
typedef struct {
  int32_t nq;
  int32_t ngates;
  int64_t state_off; /* in qcw_c64 elements */
  int64_t gate_off;  /* index of the first gate */
} qcw_instance;

typedef struct qcw_batch qcw_batch;

int qcw_batch_create(qcw_batch **out, const qcw_instance *inst, int n,
                     const qcw_gate *gates, int64_t ngates_total, const qcw_c64 *mats,
                     int64_t nmats, qcw_c64 *states, int64_t nstates,
                     const char *tune_table, void *stream);
int qcw_batch_run(qcw_batch *b, void *stream);
/* The same work enqueued directly (no graph), e.g. inside a caller's capture. */
int qcw_batch_run_eager(qcw_batch *b, void *stream);
/* The batch `reps` times in a row (1 <= reps <= 1024) with one graph launch:
 * every instance's circuit applied reps times, as reps calls of qcw_batch_run
 * would, bit for bit, for callers that step the same instances repeatedly
 * (the multiverse paths of §5 advance step after step).  The graph of reps
 * executions is captured on first use (on a private stream, which it
 * synchronises) and kept with the handle.  A graph launch costs the host
 * tens of microseconds in the HIP runtime, more than one execution of a
 * small batch takes on the device; one launch per reps executions spreads
 * that cost. */
int qcw_batch_run_repeat(qcw_batch *b, int reps, void *stream);
/* Launch shape: tile-shape variant used for instances of nq qubits, grid
 * blocks and dynamic LDS bytes per block.  Any output pointer may be NULL. */
int qcw_batch_info(const qcw_batch *b, int nq, int *variant, int *blocks, int *lds_bytes);
int qcw_batch_destroy(qcw_batch *b);
/* Name of a tile-shape variant ("amp8_sgpr", ...), as used in tune tables. */
const char *qcw_batch_variant_name(int variant);

/*
 * Gate fusion (§2c, tensor-product structure; gates compose in list order):
 * gates whose targets together span at most max_qubits (1..3) qubits become
 * one gate on that union, its matrix the product of the block's gates, each
 * extended by the identity (the first gate rightmost).  A block starts at
 * the first gate not yet placed and scans onward.  regroup = 0: the block is
 * a run of consecutive gates (gates are never reordered).  regroup = 1: a
 * gate may also join the block ahead of gates the scan passed over, provided
 * it shares no qubit with any of them (they commute, so the circuit's
 * operator is unchanged); random 36-gate circuits on 9 qubits fuse to ~13
 * gates instead of ~19.  The union's qubits are listed in order of first
 * appearance (first = most significant local bit).  A block of one gate is
 * copied unchanged; a fused matrix carries the rounding of its products, so
 * the fused circuit equals the original to FP64 rounding.
 * All arrays are host memory: gates (ngates) and mats (nmats) as for
 * qcw_circuit; out_gates must hold ngates entries, out_mats out_mats_cap
 * (64 * ngates always suffices).  Writes the fused gate count and matrix
 * entries to *out_ngates and *out_nmats.  QCW_EINVAL for an invalid gate or
 * too small an out_mats.
 */
int qcw_fuse_circuit(int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
                     int64_t nmats, int max_qubits, int regroup, qcw_gate *out_gates,
                     int *out_ngates, qcw_c64 *out_mats, int64_t out_mats_cap,
                     int64_t *out_nmats);

/*
 * Autotuner: for every qubit count in [nq_lo, nq_hi] (1 <= nq_lo <= nq_hi <=
 * 11) times one persistent launch over `ninst` synthetic instances of that
 * size (random circuits of gates_per_qubit * nq dense unitaries), once per
 * tile-shape variant, and writes the fastest variant per size to out_path.
 * Synchronises `stream`.
 */
int qcw_batch_autotune(const char *out_path, int nq_lo, int nq_hi, int ninst,
                       int gates_per_qubit, void *stream);

/*
 * Multiverse density-matrix step (§5, "The multiverse approach").
 *
 * rho is a DEVICE array of 2^nq x 2^nq qcw_c64 (nq <= 17), row-major:
 * element (n, m) = <n|rho|m> at n * 2^nq + m.  Read as a vector it is a
 * 2nq-qubit state whose qubits 1..nq are the row qubits and nq+1..2nq the
 * column qubits.
 *
 * qcw_rho_conjugate: rho <- U rho U^dagger for a k-qubit algorithm gate (the
 * Omega_A factors of Eq. rhoE4): the one-gate sweep of U on the row targets,
 * then of conj(U) on the column targets; from nq = 5 both in one pass over
 * rho (LDS tiles), with the same result bit for bit.
 *
 * A channel is the ensemble average over noisy paths, Eq. rhoE1:
 *     rho_out = p_keep * rho_in + sum_t weight_t K_t rho_in K_t^dagger,
 * where path t's operator K_t is one 2 x 2 operator on qubit q[0] (nops = 1,
 * a single hit) or the product of two 2 x 2 operators on distinct qubits q[0],
 * q[1] (nops = 2, a double hit).  In Eq. rhoE4 the weight of a path is
 * eps * p_s / n_p and p_keep = 1 - eps (the paper's p; the printed equation
 * omits it, but its trace then exceeds 1, while Eq. rhoE1 and the trace
 * argument that follows it keep it).  The operators are fixed once drawn
 * (§5, caption of the denE listing), so a channel is created once, copied to
 * the device, and applied at every step.  rho_in and rho_out must not overlap.
 * Applications of one channel must not run at the same time (on two streams
 * without an order between them): the tiled kernel keeps its work counters
 * in the channel.
 *
 * qcw_channel_create is synchronous and uses the current device, on which
 * the channel must then be applied.  For a channel whose terms are all
 * diagonal or anti-diagonal operators and 7 <= nq <= 15, it plans the tiled
 * kernel and compiles that kernel for the plan at run time (hipRTC of the
 * ROCm installation the library was built with).  The first channel of a
 * given structure (qubits and operator pattern; the coefficients and p_keep
 * do not count) takes about a second; later ones reuse the code object,
 * which stays loaded until the process ends.  Without a run-time compiler the
 * channel runs the generic tiled kernel, with the same results.
 *
 * qcw_rho_observables (synchronous) writes to out_host, 4 + 3 nq doubles:
 * Tr rho (re, im); Tr rho^2 as sum |rho_nm|^2 (equal for Hermitian rho); the
 * fidelity Tr sqrt(sqrt(rho0) rho sqrt(rho0)) = sqrt(<psi0|rho|psi0>) against
 * the pure reference rho0 = |psi0><psi0| (psi0_host: 2^nq host amplitudes, or
 * NULL, then NaN); and for qubit q = 1..nq the polarisation Tr[sigma_x,y,z^(q)
 * rho] (§5, the ideal and noisy channels).  It keeps a device scratch buffer
 * per device (about 2 MB, allocated on the first call and kept) and
 * serialises concurrent calls on it.
 */
typedef struct {
  int32_t nops;   /* 1 or 2 */
  int32_t q[2];   /* qubits, 1-based */
  int32_t pad;
  int64_t mat[2]; /* offsets of the 2 x 2 operators in mats */
  double weight;
} qcw_kraus_term;

typedef struct qcw_channel qcw_channel;

int qcw_rho_conjugate(int k, const int *targets, const qcw_c64 *U, qcw_c64 *rho, int nq,
                      void *stream);
int qcw_channel_create(qcw_channel **out, int nq, double p_keep, const qcw_kraus_term *terms,
                       int nterms, const qcw_c64 *mats, int64_t nmats);
int qcw_channel_apply(const qcw_channel *c, const qcw_c64 *rho_in, qcw_c64 *rho_out,
                      void *stream);
/*
 * One multiverse step of Eq. rhoE4 in one call:
 *     rho_out = U [channel(rho_in)] U^dagger
 * for a k-qubit algorithm gate U on the targets (conventions of qcw_opk).
 * When U is monomial, U |l> = u_l |pi(l)> (one nonzero entry in each row
 * and column: X, CNOT, SWAP, Toffoli, Z, S, T, Y, CZ, ...), and the channel
 * runs its compiled tiled kernel, the conjugation is folded into that
 * kernel: output (n, m), times u_l(n) conj(u_l(m)), is stored at
 * (pi(n), pi(m)), one pass over rho instead of two.  Any other gate whose
 * targets are all among the four last qubits (nq - 3 .. nq: state bits
 * 0..3, whose rows and columns each tile of the kernel holds complete) is
 * folded as well: the kernel applies U to the rows and conj(U) to the
 * columns of each tile's outputs in LDS, with the same operations as
 * qcw_rho_conjugate, and U is passed with the launch.  The kernel for each
 * such gate (for the latter, each target list) is compiled on its first use
 * (under a second, synchronous).
 * Otherwise it is qcw_channel_apply followed by qcw_rho_conjugate on rho_out.
 * Either way the result is the same, bit for bit up to the sign of zeros.
 * rho_in and rho_out must not overlap.
 */
int qcw_channel_apply_gate(const qcw_channel *c, const qcw_c64 *rho_in, qcw_c64 *rho_out, int k,
                           const int *targets, const qcw_c64 *U, void *stream);
/*
 * The same step (k = 0: the channel alone), also reducing the new rho's
 * observables of §5 into obs (DEVICE, 4 + 3 nq doubles, written
 * asynchronously on stream), laid out as qcw_rho_observables: Tr rho (re,
 * im), Tr rho^2 as sum |rho_nm|^2, the root fidelity sqrt(<psi0|rho|psi0>)
 * against psi0 (DEVICE, 2^nq amplitudes; NULL: NaN), and each qubit's
 * polarisation.  When the step runs as the compiled kernel (a gate folded as
 * above, or none), that kernel sums the first four as it stores rho, with no
 * further pass over rho; the polarisations read the 2 x 2 blocks on each
 * qubit afterwards.  Otherwise the step is followed by the observables
 * kernels.  The sums run in an order fixed by nq, so
 * repeated calls give the same bits.  The channel keeps a partial-sum buffer
 * (allocated on first use, up to 128 MB at nq = 15): steps of one channel
 * must not run at the same time.  The first call may synchronise the device
 * (to replace that buffer); later calls do not.
 */
int qcw_channel_step_obs(qcw_channel *c, const qcw_c64 *rho_in, qcw_c64 *rho_out, int k,
                         const int *targets, const qcw_c64 *U, const qcw_c64 *psi0,
                         double *obs, void *stream);
int qcw_channel_destroy(qcw_channel *c);
/* Real FP64 operations per output element of one application, as evaluated
 * by the kernel the channel runs (for roofline accounting).  Terms whose
 * operators are all diagonal or anti-diagonal (Pauli operators, phases, the
 * identity) read rho at n^x, m^x for a flip mask x, and terms with equal
 * masks share that read.
 * - Tiled kernel (every term of that kind, 7 <= nq <= 15): the coefficients
 *   of a mask group are summed on the host into tables over the group's
 *   qubits (segments of at most three qubits), so a group costs one
 *   multiply-add with its coefficient, 4 when every coefficient is real
 *   (Pauli channels) and 8 otherwise, plus 1 (real) or 2 per further segment.
 * - Gather kernel (otherwise): 8 per mask group, plus 2 per one-operator
 *   term and 8 per two-operator term for its coefficient; any other term
 *   costs 8 per complex multiply-add (4 for one operator, 16 for two) plus 4
 *   for its weighted sum.
 * Plus 2 for p_keep * rho. */
int64_t qcw_channel_flops_per_element(const qcw_channel *c);

/*
 * The plan of a channel's tiled kernel, and the choice of kernel (host call,
 * for tests).  kernel: from now on, 0 runs the tiled kernel when there is a
 * plan (the one compiled for this channel at creation when the run-time
 * compiler gave one, else the generic tiled kernel), 1 the gather kernel,
 * 2 the generic tiled kernel; negative leaves the choice.  Both tiled kernels
 * give the same bits.  info (17 host int32): {has tiled plan, kernel in use
 * (0 tiled, 1 gather), tile bits E0, E1, partner tiles (with the tile
 * itself), partners staged in LDS, partners read directly, tile itself
 * staged, read sets, mask groups, segments, segments on E0 or E1, all
 * coefficients real, the compiled tiled kernel in use, workgroups and VGPRs
 * per lane of the tiled kernel in use (0 for the gather kernel), version of
 * the run-time compiler that built the compiled kernel (major * 100 + minor;
 * 0 when there is none)}.  The run-time compiler is the hipRTC of the ROCm
 * installation the library was built with, loaded in a link-map namespace of
 * its own, so that another hipRTC already in the process (a PyTorch wheel
 * bundles one) is not the one used.  QCW_EINVAL for NULL or a kernel choice
 * above 2.
 */
int qcw_debug_channel_plan(qcw_channel *c, int kernel, int32_t *info);

/*
 * The source of the tiled kernel that qcw_channel_create would compile for
 * these terms (host call, no device needed; for tests).  Arguments as for
 * qcw_channel_create; gate_k != 0 asks instead for the kernel that
 * qcw_channel_apply_gate compiles for the gate (gate_k, gate_targets, gate_U),
 * which has none (length 0) unless the gate is monomial or has every target
 * among the four last qubits; observables != 0
 * asks for the variant of qcw_channel_step_obs, which also sums them.  *len:
 * the source's length (0 when the channel has no tiled plan); when buf is
 * not NULL, up to cap - 1 bytes of it and a NUL are written there.  compile != 0: the source is also compiled for gfx950 with
 * the run-time compiler and *code_bytes set to the code object's size; a
 * failed compile returns QCW_EHIP with the compiler's log in the last error.
 * compiler_version (may be NULL): the run-time compiler's version, major *
 * 100 + minor, 0 when it cannot be loaded.  QCW_EINVAL for bad terms or NULL
 * len (or code_bytes when compiling).
 */
int qcw_debug_channel_source(int nq, const qcw_kraus_term *terms, int nterms, const qcw_c64 *mats,
                             int64_t nmats, int gate_k, const int *gate_targets,
                             const qcw_c64 *gate_U, int observables, int compile, char *buf,
                             size_t cap, size_t *len, size_t *code_bytes,
                             int32_t *compiler_version);
int qcw_rho_observables(const qcw_c64 *rho, int nq, const qcw_c64 *psi0_host,
                        double *out_host, void *stream);
/*
 * The 15 parameters of two qubits qa and qb (1-based, distinct) of rho, in
 * the two-qubit form of the footnote to §5's density-matrix paragraph,
 *   rho_ab = (1 + P1 . (sigma x 1) + P2 . (1 x sigma) + C . (sigma x sigma)) / 4,
 * rho_ab being the reduced density matrix of (qa, qb) in that order: out
 * (DEVICE, 15 doubles) gets P1 = Tr[(sigma x 1) rho] (x, y, z), P2 =
 * Tr[(1 x sigma) rho], and the spin correlation tensor C_ij = Tr[(sigma_i x
 * sigma_j) rho], row-major (i for qa).  The footnote's traces omit rho; they
 * are read as in the one-qubit case P = Tr[sigma rho] before it.  P1 is
 * qa's polarisation from qcw_rho_observables (to rounding).  Asynchronous on
 * stream, sums in an order fixed by nq.  QCW_EINVAL for nq outside [2, 17]
 * or bad qubits.
 */
int qcw_rho_pair_polarization(const qcw_c64 *rho, int nq, int qa, int qb, double *out,
                              void *stream);

/*
 * Eigenvalue-based observables (§5, classical-limit discussion: the paper
 * follows entropy, purity, fidelity and the eigenvalues of rho at every stage),
 * for nq <= 6 (a 64 x 64 rho; the paper's examples use 1, 2 and 5 qubits), by
 * a parallel cyclic Jacobi eigensolver, one workgroup per matrix with the
 * matrix in LDS.  Every call takes the Hermitian part (rho + rho^dagger) / 2.
 *
 * qcw_rho_eigvals_batch: `count` matrices, matrix i at rho + i * stride
 * (device, stride >= 4^nq elements); writes the eigenvalues of matrix i in
 * ascending order to eig[i * 2^nq ...] (device, count * 2^nq doubles) and the
 * von Neumann entropy -sum lambda log2 lambda in bits (over lambda > 0; it
 * tends to nq in the classical limit; the paper writes S = -Tr rho ln rho, and
 * the value in nats is the bits value times ln 2) to entropy[i] (device, count
 * doubles, or NULL).  One persistent launch on `stream`: asynchronous, no
 * device memory allocated, no synchronisation.  Eigenvalues agree with a
 * Hermitian LAPACK solver to ~1e-15 (absolute, trace-one rho).
 *
 * qcw_rho_fidelity_batch: F_i = Tr sqrt(sqrt(rho0_i) rho_i sqrt(rho0_i)), the
 * root fidelity (1/sqrt2 after one Hadamard on |0>, §5), for pairs rho_i =
 * rho + i * rho_stride, rho0_i = rho0 + i * rho0_stride (rho0_stride = 0: one
 * reference for all); fidelity: device, count doubles.  Asynchronous, no
 * allocation.  It is evaluated on the range of rho0: with rho0's eigenvalues
 * l above n * eps * l_max and their eigenvectors V_r, F = Tr sqrt(K) for the
 * r x r matrix K = diag(sqrt l) V_r^dagger rho V_r diag(sqrt l), whose nonzero
 * eigenvalues are those of sqrt(rho0) rho sqrt(rho0); eigenvalues of K at or
 * below r * eps * max(K) are taken as zero.  A pure reference gives r = 1 and
 * F = sqrt(<psi0|rho|psi0>).  Accuracy ~1e-15 when K's eigenvalues are
 * either rounding-level or well above it; the definition itself is
 * ill-conditioned at rank-deficient inputs (the square root of an eigenvalue
 * d moves by d / (2 sqrt d)), so an input perturbed at the rounding level
 * can move F by ~sqrt(eps) ~ 1e-8 through eigenvalues just above the cut.
 *
 * qcw_rho_eigvals and qcw_rho_fidelity are the same for one matrix with host
 * outputs (synchronous): qcw_rho_eigvals writes 2^nq + 1 doubles to out_host
 * (the eigenvalues ascending, then the entropy in bits); qcw_rho_fidelity
 * writes F.  They share a small device buffer per device, allocated on first
 * use and kept, and serialise on it.
 * qcw_rho_partial_trace (asynchronous) writes the reduced density matrix of
 * the nkeep qubits keep[] (1-based, distinct) to the device array out
 * (2^nkeep x 2^nkeep, the lowest-numbered kept qubit most significant), for
 * subsystem entropies and eigenvalues.
 */
int qcw_rho_eigvals_batch(const qcw_c64 *rho, int nq, int64_t count, int64_t stride, double *eig,
                          double *entropy, void *stream);
int qcw_rho_fidelity_batch(const qcw_c64 *rho, int64_t rho_stride, const qcw_c64 *rho0,
                           int64_t rho0_stride, int nq, int64_t count, double *fidelity,
                           void *stream);
int qcw_rho_eigvals(const qcw_c64 *rho, int nq, double *out_host, void *stream);
int qcw_rho_fidelity(const qcw_c64 *rho, const qcw_c64 *rho0, int nq, double *out_host,
                     void *stream);
int qcw_rho_partial_trace(const qcw_c64 *rho, int nq, const int *keep, int nkeep, qcw_c64 *out,
                          void *stream);

/*
 * Serving: a continuous-batching request loop on one GPU.  Requests (one
 * instance each: a state of nq <= cfg.max_nq <= 11 qubits and its circuit)
 * are submitted from any thread; a scheduler thread admits them in arrival
 * order whenever a slot and enough of the device-memory budget are free,
 * keeps each admitted state resident in device memory until its circuit is
 * done, and runs ticks: one persistent batch launch that advances every
 * resident request by up to gates_per_tick gates (0 = all remaining gates).
 * Requests that arrive while a tick runs join the next tick.  A request
 * never leaves the queue except by completing or failing, and the queue head
 * is never overtaken (no starvation).  Results equal, bit for bit, those of
 * qcw_circuit run on the request alone, unless the tune table puts the
 * request's size on "amp4_mfma" (see qcw_batch_create): then the request's
 * circuit is fused at submit and results agree to FP64 rounding.
 *
 * All request arrays are HOST pointers copied by qcw_server_submit, which
 * does not block on the GPU.  Uploads and result copies are batched per
 * tick: beside the arena the server holds a staging buffer of 64 MiB (or the
 * budget, if smaller) and a result buffer of min(budget, max_slots * 16 *
 * 2^max_nq) bytes, each on the device and in pinned host memory.  A request
 * that can never run (invalid gates,
 * nq above the limit, more memory than the whole budget) is rejected with
 * QCW_EINVAL at submit and affects no other request.
 */
typedef struct {
  uint64_t hbm_budget_bytes; /* device arena for resident requests */
  int max_slots;             /* most requests resident at once */
  int gates_per_tick;        /* 0: run all remaining gates in one tick */
  int max_nq;                /* largest request size, <= 11 */
  const char *tune_table;    /* NULL: built-in tile shapes */
} qcw_server_cfg;

typedef struct {
  int nq;
  int ngates;
  const qcw_gate *gates; /* matrix offsets relative to mats */
  const qcw_c64 *mats;
  int64_t nmats;
  const qcw_c64 *psi0; /* 2^nq amplitudes */
} qcw_request;

typedef struct {
  int status;          /* QCW_OK, QCW_EAGAIN (pending) or an error */
  int ticks;           /* ticks the request was resident for */
  uint64_t t_submit_ns; /* CLOCK_MONOTONIC nanoseconds */
  uint64_t t_admit_ns;
  uint64_t t_done_ns;
} qcw_req_stats;

typedef struct {
  uint64_t submitted, completed, rejected, ticks;
  uint64_t peak_active, peak_pending, admit_waits;
} qcw_server_counters;

typedef struct qcw_server qcw_server;

int qcw_server_create(qcw_server **out, const qcw_server_cfg *cfg);
int qcw_server_submit(qcw_server *s, const qcw_request *r, uint64_t *ticket);
/* QCW_OK: finished; the final state is copied to psi_out_host (may be NULL)
 * and the ticket is released.  QCW_EAGAIN: still pending.  Another code: the
 * request failed or the ticket is unknown.  st may be NULL. */
int qcw_server_poll(qcw_server *s, uint64_t ticket, qcw_c64 *psi_out_host,
                    qcw_req_stats *st);
/* As poll, but blocks up to timeout_s seconds for completion. */
int qcw_server_wait(qcw_server *s, uint64_t ticket, qcw_c64 *psi_out_host,
                    qcw_req_stats *st, double timeout_s);
int qcw_server_counters_get(qcw_server *s, qcw_server_counters *out);
/* Stops the scheduler after the current tick; pending requests fail. */
int qcw_server_destroy(qcw_server *s);

/*
 * Kernel timing.  While enabled, every kernel the library launches is
 * bracketed by HIP events recorded on the stream it is launched on.
 * qcw_timing_read synchronises those events and returns, for one kernel
 * family, the number of launches and their summed duration in milliseconds
 * since the last reset.  Families: QCW_KERNEL_SWEEP1..3 (one-gate sweeps of
 * k = 1, 2, 3, in either sweep kernel), QCW_KERNEL_BATCH (batch executions),
 * QCW_KERNEL_FUSED (fused passes), QCW_KERNEL_CHANNEL (channel applications,
 * with or without a folded permutation gate), QCW_KERNEL_SMALL (launches of
 * qcw_circuit on states of at most 11 qubits), QCW_KERNEL_CONJ (one-pass
 * conjugations of qcw_rho_conjugate).
 * Launches recorded into a hipGraph are not timed individually.
 */
enum {
  QCW_KERNEL_SWEEP1 = 1,
  QCW_KERNEL_SWEEP2 = 2,
  QCW_KERNEL_SWEEP3 = 3,
  QCW_KERNEL_BATCH = 4, /* one batch execution (qcw_batch_run: the graph) */
  QCW_KERNEL_FUSED = 5, /* one fused pass */
  QCW_KERNEL_CHANNEL = 6, /* one channel application */
  QCW_KERNEL_SMALL = 7,   /* one launch of qcw_circuit on a state of <= 11 qubits */
  QCW_KERNEL_CONJ = 8,    /* one one-pass conjugation rho <- U rho U^dagger */
  QCW_KERNEL_COUNT = 9
};
int qcw_timing_enable(int on);
int qcw_timing_reset(void);
int qcw_timing_read(int kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* QCW_H */
