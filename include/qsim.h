/*
 * qsim.h -- C ABI of the MI355X (gfx950) full-amplitude state-vector library.
 *
 * The calls follow the problem statement of the paper (Zhong, Fan, Li,
 * "Scalable Parallel Simulation of Quantum Circuits on CPU and GPU Systems"):
 *   - a state is 2^n complex amplitudes, index bit q <-> qubit q
 *     (Section 2.1, Eq. 1 and Eq. 2);
 *   - a circuit is a time-ordered gate list applied to the state
 *     (Section 2.1, Eq. 3 and Eq. 4; Section 2.2, Algorithms 1-4);
 *   - gates are contracted into k-qubit unitaries along a dependency DAG
 *     (Section 3.4, Eq. 6 and the Kronecker-fusion equations);
 *   - energies are expectations of Pauli sums (Section 1, VQE).
 *
 * Conventions for every call:
 *   - Every function returns a qs_status; nothing throws across the ABI.
 *     On failure qs_last_error() returns a thread-local message.
 *   - Host arrays passed in are owned by the caller and only read during
 *     the call.  Plans and batches are owned by the library until their
 *     *_destroy call.  State memory given as dev_ptr stays caller-owned.
 *   - Device work is ordered on the stream given to qs_state_create (or the
 *     batch).  Functions that return host values synchronise that stream.
 *   - All compute runs in the library's HIP kernels; there is no CPU
 *     fallback.  Without a usable gfx950 device the device calls return
 *     QS_EDEVICE.  Host-only calls (qs_contract, qs_plan_*) work anywhere,
 *     except qs_contract with QS_STRATEGY_LEARNED and a loaded cost model:
 *     it runs the model's inference kernel, so it needs the device that
 *     holds the model (without a model that strategy is plain greedy and
 *     stays host-only).
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QS_OK = 0,
    QS_EINVAL = -1,        /* bad argument: qubit out of range, duplicate qubit, null pointer, ... */
    QS_ENOMEM = -2,        /* device or host allocation failed */
    QS_EDEVICE = -3,       /* HIP runtime error or no usable device */
    QS_ERANGE = -4,        /* size beyond a documented limit */
    QS_EUNSUPPORTED = -5   /* valid request this build does not implement */
} qs_status;

/* Amplitude storage: interleaved (re, im) complex64 (8 B) or complex128 (16 B). */
typedef enum { QS_C64 = 0, QS_C128 = 1 } qs_dtype;

/* Gate kinds.  Matrices (row-major, <r|U|c>):
 *   H = [[1,1],[1,-1]]/sqrt2, X, Y = [[0,-i],[i,0]], Z, S = diag(1,i), SDG,
 *   T = diag(1,e^{i pi/4}), TDG, RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2),
 *   RZ(t) = diag(e^{-it/2}, e^{it/2}), P(l) = diag(1, e^{il}),
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]].
 * Controlled kinds (qubits[0] = control, qubits[1] = target) act as
 * |0><0| (x) I + |1><1| (x) U with U = X (CNOT), Z (CZ), P(l) (CP), U3 (CU)
 * (Section 2.1, Eq. 4).  SWAP exchanges two qubits.  DENSE is a k-qubit
 * matrix (1 <= k <= 6) given in `matrix` with local bit j <-> qubits[j]. */
typedef enum {
    QS_H = 0, QS_X, QS_Y, QS_Z, QS_S, QS_SDG, QS_T, QS_TDG,
    QS_RX, QS_RY, QS_RZ, QS_U3, QS_P,
    QS_CNOT, QS_CZ, QS_CP, QS_CU, QS_SWAP, QS_DENSE,
    QS_NUM_KINDS
} qs_kind;

/* One gate; 80 bytes.  params[0..2] = (theta, phi, lambda) where used.
 * matrix: only for QS_DENSE, 2^nq x 2^nq complex128, interleaved re/im,
 * row-major; read during the call that receives the gate list. */
typedef struct {
    int32_t kind;
    int32_t nq;
    int32_t qubits[8];
    double params[4];
    const double *matrix;
} qs_gate;

typedef struct qs_state_s *qs_state;
typedef struct qs_plan_s *qs_plan;
typedef struct qs_batch_s *qs_batch;

/* Contraction strategies (Section 3.4). */
enum {
    QS_STRATEGY_NONE = 0,    /* one block per gate, still streamed in tile passes */
    QS_STRATEGY_GREEDY = 1,  /* fixed-width greedy merge over the DAG (width k_max) */
    QS_STRATEGY_LEARNED = 2, /* widths chosen per pass by the loaded cost model; greedy if none loaded */
    QS_STRATEGY_PAULI = 3    /* greedy, after contracting every run of gates that multiplies to one
                                Pauli rotation exp(-i phi P) (Clifford gates around one diagonal
                                one-qubit gate, Clifford parts cancelling, X support <= 8 qubits
                                and < tile_qubits) into one block; beyond Section 3.4's rule */
};

typedef struct {
    int32_t k_max;        /* largest fused block, 1..6 (complex128: 1..5); 0 = 5 */
    int32_t tile_qubits;  /* t: qubits held per tile in LDS; 0 = auto (13 for c64, 12 for c128) */
    int32_t low_qubits;   /* c: qubits 0..c-1 always in the tile (contiguous run); 0 = auto (6) */
    int32_t strategy;     /* QS_STRATEGY_* */
    int32_t renorm;       /* 1: FP64 norm of every pass, next pass rescales by 1/sqrt(norm) */
    int32_t dtype;        /* qs_dtype the plan is costed for (learned strategy); default c64 */
    int32_t commute;      /* 1: a gate may be contracted past earlier gates it commutes with, i.e.
                             gates diagonal (commuting with Z) on every qubit they share, such as
                             phase and CZ gates with each other or with a CNOT's control; 0: every
                             pair of gates sharing a qubit keeps its order (Section 3.4's DAG).
                             Applies to the greedy contraction of every strategy. */
    int32_t reserved;
} qs_contract_opts;

typedef struct {
    int32_t n;            /* qubits */
    int32_t max_k;        /* widest block */
    uint64_t n_gates;     /* gates in the circuit */
    uint64_t n_blocks;    /* fused blocks */
    uint64_t n_passes;    /* streamed passes over the state */
    uint64_t blocks_by_k[8];  /* blocks_by_k[k] = number of blocks of width k (k <= 7) */
    double flops_per_amp; /* sum over blocks of 8 * 2^k real flops per amplitude */
} qs_plan_info;

/* ----------------------------------------------------------- library */
const char *qs_last_error(void);
const char *qs_version(void);

/* Current HIP device: compute units, LDS bytes per workgroup, gfx arch name
 * (writes at most arch_len bytes including the terminating 0). */
qs_status qs_device_query(int *cu_count, int *lds_bytes, char *arch, size_t arch_len);

/* -------------------------------------------------------------- state */
/* Create a state of n qubits (1 <= n <= 40).  dev_ptr: caller-owned device
 * buffer of 2^n amplitudes of `dtype` (16-byte aligned), or NULL for a
 * library-owned allocation.  stream: hipStream_t (NULL = default stream).
 * The amplitudes are not initialised; call qs_state_set_basis. */
qs_status qs_state_create(int n, qs_dtype dtype, void *dev_ptr, void *stream, qs_state *out);
qs_status qs_state_destroy(qs_state s);   /* never frees caller-owned memory */
qs_status qs_state_data(qs_state s, void **dev_ptr);
/* |index> (Eq. 1 with alpha_index = 1).  index < 2^n. */
qs_status qs_state_set_basis(qs_state s, uint64_t index);
/* Apply a pending per-pass renormalisation to the stored amplitudes (one sweep).
 * Passes leave the last pass's scale pending; reads below account for it. */
qs_status qs_state_normalize(qs_state s);
/* Copy `count` amplitudes starting at `offset` to host memory as interleaved
 * FP64 (re, im) pairs, with any pending renormalisation applied.  Synchronous. */
qs_status qs_state_copy_out(qs_state s, uint64_t offset, uint64_t count, double *host);
/* Copy amplitudes in from interleaved FP64 host memory (rounded to the
 * state's dtype).  Synchronous. */
qs_status qs_state_copy_in(qs_state s, uint64_t offset, uint64_t count, const double *host);
/* FP64 sum of |psi_i|^2 of the state as read by qs_state_copy_out. Synchronous. */
qs_status qs_norm(qs_state s, double *out);

/* ------------------------------------------------- plain gate-by-gate */
/* Apply gates in program order, one HIP kernel sweep per gate (Algorithms 1
 * and 2; controlled gates touch only the control-1 half, Eq. 4).  The list
 * is validated before anything is launched: any bad gate -> QS_EINVAL and
 * the state is unchanged.  Asynchronous on the state's stream. */
qs_status qs_apply_gates(qs_state s, const qs_gate *gates, size_t n_gates);

/* The same circuit with staggered multi-gate parallelism (Section 3.3, the
 * two-dimensional thread mapping and Table "segment"): the gates are grouped
 * into DAG layers (gates of a layer share no qubit); the one-qubit and
 * controlled one-qubit gates of a layer, up to 32 at a time, run in 2^s launches
 * over 2^s state segments chosen by s qubits none of them touches, gate i
 * updating segment (i + j) mod 2^s at step j; other gates run as in
 * qs_apply_gates.  Every gate still sweeps the amplitudes it touches once.
 * Same state as qs_apply_gates up to rounding order; validation, errors and
 * asynchrony as there. */
qs_status qs_apply_gates_smgp(qs_state s, const qs_gate *gates, size_t n_gates);

/* -------------------------------------------------- contraction (host) */
/* Build a plan for an n-qubit circuit: the dependency DAG of Section 3.4
 * (gates sharing a qubit keep program order; with opts->commute, gates and
 * blocks that are diagonal on every qubit they share may pass each other, as
 * may Pauli-rotation blocks whose strings commute), blocks merged under the
 * chosen strategy with FP64 block products, and blocks packed into tile
 * passes.  Host only, except the learned strategy, which evaluates the cost
 * model on the current device.  opts may be NULL (defaults).  The commute
 * option's greedy rule scans the blocks a gate may join, O(gates x blocks)
 * in the worst case (many mutually commuting gates). */
qs_status qs_contract(int n, const qs_gate *gates, size_t n_gates,
                      const qs_contract_opts *opts, qs_plan *out);
qs_status qs_plan_destroy(qs_plan p);
qs_status qs_plan_info_get(qs_plan p, qs_plan_info *info);
/* Block b: width k, its qubits ascending (k entries), its FP64 matrix
 * (4^k complex, interleaved, row-major, local bit j <-> j-th smallest qubit;
 * NULL to skip; QS_EUNSUPPORTED for Pauli-rotation blocks wider than 10
 * qubits), and its member gate indices in program order (member_cap entries
 * at most; *n_members gets the true count).  k may exceed k_max for blocks of
 * the Pauli strategy (up to 8 + the Z part of the rotation). */
qs_status qs_plan_block(qs_plan p, uint64_t b, int *k, int *qubits, double *matrix,
                        uint64_t *members, uint64_t member_cap, uint64_t *n_members);
/* Pass i: tile width t, its tile qubits ascending (t entries), first block
 * index and block count. */
qs_status qs_plan_pass(qs_plan p, uint64_t i, int *t, int *tile_qubits,
                       uint64_t *first_block, uint64_t *n_blocks);
/* Run a plan on a state (same n): one tile-pass kernel per pass.
 * Asynchronous on the state's stream. */
qs_status qs_apply_plan(qs_state s, qs_plan p);

/* ------------------------------------------------------- expectation */
/* Energy sum_k coeff[k] <psi|P_k|psi> / <psi|psi> of a Pauli sum; P_k has X or
 * Y on the set bits of x[k], Z or Y on the set bits of z[k] (Y where both).
 * FP64 accumulation; out_terms (optional, n_terms entries) receives each
 * <P_k>.  Synchronous. */
qs_status qs_expect_pauli_sum(qs_state s, const uint64_t *x, const uint64_t *z,
                              const double *coeff, size_t n_terms, double *out,
                              double *out_terms);
/* The same energy for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * device memory is allocated or freed; the kernels' tables, per-workgroup
 * partials and results live in a device array the library holds per GPU
 * until the process ends (about 5 MiB).  At most 2048 terms per call
 * (QS_ERANGE above).  Calls in one process take turns on a GPU's array (a
 * lock), and every call leaves the array's contents behind for the next one,
 * which overwrites what it reads.  Same arguments, results and
 * synchronisation as qs_expect_pauli_sum. */
qs_status qs_expect_pauli_sum_noalloc(qs_state s, const uint64_t *x, const uint64_t *z,
                                      const double *coeff, size_t n_terms, double *out,
                                      double *out_terms);

/* ------------------------------------------------------------ batches */
/* A batch of independent states (uneven qubit counts, 1 <= n_i <= 26),
 * each with its circuit and Pauli-sum Hamiltonian, run by ONE persistent
 * kernel captured in a hipGraph.  Plans use opts (NULL = defaults; a zero
 * k_max/tile asks the autotuner).  State memory is library-owned. */
qs_status qs_batch_create(int n_states, const int *n_qubits, const qs_gate *const *circuits,
                          const size_t *n_gates, const uint64_t *const *x, const uint64_t *const *z,
                          const double *const *coeff, const size_t *n_terms,
                          const qs_contract_opts *opts, void *stream, qs_batch *out);
qs_status qs_batch_destroy(qs_batch b);
/* Reset every state to |0..0>, run all circuits and energies with one graph
 * launch; energies[i] receives state i's energy.  Synchronous. */
qs_status qs_batch_run(qs_batch b, double *energies);
/* Copy state i's amplitudes (normalised, FP64 interleaved) to the host. */
qs_status qs_batch_state_copy_out(qs_batch b, int i, double *host);

/* -------------------------------------------------------------- tuning */
/* Time candidate (k_max, tile_qubits, low_qubits) triples for this circuit
 * on the device and return the fastest in *best (strategy and renorm copied
 * from base).  The circuit (its first 1536 gates when longer) runs on a
 * scratch state of its own size.  Synchronous. */
qs_status qs_autotune(int n, qs_dtype dtype, const qs_gate *gates, size_t n_gates,
                      const qs_contract_opts *base, qs_contract_opts *best);

/* ---------------------------------------------------------- cost model */
/* Number of features per pass candidate. */
int qs_costmodel_num_features(void);
/* Features of every pass of a plan (rows of qs_costmodel_num_features()). */
qs_status qs_plan_pass_features(qs_plan p, float *out, uint64_t cap_rows);
/* Device timing of every pass of a plan on a scratch state; us_out[i] is the
 * median of `reps` hipEvent-timed launches of pass i.  Synchronous. */
qs_status qs_plan_time_passes(qs_plan p, qs_dtype dtype, int reps, double *us_out);
/* Train the MLP (F -> h1 -> h2 -> 1, ReLU) on (features, log-microseconds)
 * with the library's forward/backward/Adam kernels on the device.  Weights
 * start from `init_weights` if not NULL.  Synchronous. */
qs_status qs_costmodel_train(const float *features, const float *targets, int n_rows,
                             int epochs, int batch, float lr, uint64_t seed,
                             const float *init_weights, float *loss_out);
/* Load / store the active model: flat FP32 weights W1,b1,W2,b2,W3,b3. */
int qs_costmodel_num_weights(void);
qs_status qs_costmodel_set_weights(const float *w);
qs_status qs_costmodel_get_weights(float *w);
/* Device inference on rows of features; out receives predicted log-us. */
qs_status qs_costmodel_predict(const float *features, int n_rows, float *out);
/* One forward+backward on the device for a batch: returns the loss and the
 * gradient (same layout as the weights).  Used to check the kernels. */
qs_status qs_costmodel_grad(const float *weights, const float *features, const float *targets,
                            int n_rows, float *grad_out, float *loss_out);

/* ------------------------------------------------------------ profiling */
/* Kernel classes timed with hipEvents when profiling is on. */
enum { QS_PROF_PLAIN = 0, QS_PROF_TILE = 1, QS_PROF_REDUCE = 2, QS_PROF_EXPECT = 3, QS_PROF_COPY = 4,
       QS_PROF_CLASSES = 5 };
typedef struct {
    uint64_t launches[QS_PROF_CLASSES];
    double ms[QS_PROF_CLASSES];        /* summed event time per class */
    double bytes[QS_PROF_CLASSES];     /* algorithmic bytes per class */
    double flops[QS_PROF_CLASSES];     /* algorithmic flops per class */
} qs_profile;
qs_status qs_profile_enable(int on);
/* Synchronise all recorded events, fill *out and reset the counters. */
qs_status qs_profile_collect(qs_profile *out);

/* Device copy of `bytes` bytes (16-byte multiple) on `stream`: the measured
 * ceiling for streaming kernels.  Asynchronous. */
qs_status qs_copy(void *dst, const void *src, uint64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
