/*
 * stn.h - C ABI of libstn, the MI355X (gfx950) hot path of the hybrid
 * stabilizer-tensor-network (STN) simulation of surface-code syndrome
 * extraction under coherent crosstalk (Harper, Nakhl, Sevior, Usman).
 *
 * The simulated state is psi = C |MPS> (Sec. IV.A, Eq. 7): a Clifford C held
 * as a bit-packed inverse tableau and a matrix-product state, for a batch of
 * independent shots that share one circuit.  Clifford gates only update the
 * tableau (Sec. IV.A); a crosstalk rotation exp(-i theta P) is rewritten
 * through the tableau into a Pauli string P' on the MPS, the MPS becomes
 * cos(theta) phi - i sin(theta) P' phi, and its bonds are cut back to chi_max
 * by keeping the largest Schmidt values (Sec. IV.A-B, Eqs. 4 and 8); a Z
 * measurement is commuted through the tableau and projected on the MPS
 * (Sec. IV.A, last paragraph).
 *
 * Conventions shared by every call:
 *  - Memory: every device buffer is owned by the caller.  The library keeps
 *    pointers into the workspace given to stn_init and never allocates device
 *    memory itself.  Pointers named dev_* are device pointers, host_* are
 *    host pointers.  All work is enqueued on the stream given in stn_config
 *    (NULL = the default stream); calls return before the work completes
 *    unless stated otherwise.
 *  - Threads: a context is used by one host thread at a time.
 *  - Errors: argument errors are detected on the host and returned at once
 *    (STN_EINVAL), leaving the context unchanged.  Errors found by kernels
 *    (an impossible forced outcome, a non-finite number, a non-converged
 *    eigen-solve) set a device error word; stn_sync, stn_logprob and the
 *    stn_get_* calls synchronise and report it.  After a device error the
 *    context state is undefined: free it.  stn_last_error gives a message.
 *  - Qubits are numbered 0..n_qubits-1 and qubit q is MPS site q.
 *  - Shot bit-masks are "sign words": uint64 words with bit (s % 64) of word
 *    (s / 64) belonging to shot s; n_sign_words = ceil(n_shots / 64).
 */
#ifndef STN_H
#define STN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stn_ctx stn_ctx;

typedef enum {
    STN_OK = 0,
    STN_EINVAL = -1,     /* bad argument (index out of range, size mismatch, ...) */
    STN_ENOMEM = -2,     /* workspace too small */
    STN_EDEVICE = -3,    /* HIP runtime error */
    STN_EZEROPROB = -4,  /* a forced measurement outcome has probability 0 */
    STN_ENUMERIC = -5,   /* NaN/Inf, odd tableau phase or eigen-solve failure */
    STN_ESTATE = -6      /* call not valid in the current state */
} stn_status;

enum { STN_FP64 = 0,   /* complex128 everywhere */
       STN_FP32 = 1 }; /* complex64 tensors and contractions; FP64 Gram,
                          eigen-solve, norms and probabilities */

typedef struct {
    int n_qubits;        /* chain length n, 1..1024 */
    int n_shots;         /* independent shots simulated together, >= 1 */
    int chi_max;         /* bond-dimension cap (Sec. IV.B), 1..1024 */
    int precision;       /* STN_FP64 or STN_FP32 */
    double eps_cut;      /* drop Schmidt values with lambda^2 <= eps_cut * sum lambda^2
                            (Eq. 8).  The squared values come from an FP64 Gram
                            eigen-solve, whose absolute error is a few FP64 epsilons
                            times sum lambda^2: cuts below ~1e-14 let rounding
                            decide the kept count.  STN_FP32, fused schedule: where
                            fewer pivots of the pivoted Cholesky factor of the
                            Gram than chi_max (and 2^min(j, n-j)) stay above
                            eps_cut * trace, those pivot rows span the kept space
                            (no eigen-solve); each direction left out then holds
                            at most eps_cut * trace. */
    void *stream;        /* hipStream_t, or NULL for the default stream */
} stn_config;

/* Gate kinds for stn_clifford.  Two-qubit kinds take (q0 = control, q1 = target). */
enum { STN_GATE_H = 0, STN_GATE_S = 1, STN_GATE_SDG = 2, STN_GATE_X = 3,
       STN_GATE_Y = 4, STN_GATE_Z = 5, STN_GATE_CX = 6, STN_GATE_CY = 7,
       STN_GATE_CZ = 8 };

typedef struct {
    int32_t kind;        /* STN_GATE_* */
    int32_t q0, q1;      /* q1 ignored (set -1) for one-qubit gates */
} stn_gate;

/* Bytes of device workspace stn_init needs for this configuration (0 on a
 * bad configuration).  The bytes cover the tableau, the MPS of every shot
 * at its largest possible bonds, the doubled-bond compression workspace and
 * per-shot scratch. */
size_t stn_workspace_bytes(const stn_config *cfg);

/* Create a context.  dev_workspace: caller-owned device memory of at least
 * stn_workspace_bytes(cfg) bytes, 256-byte aligned, kept alive until
 * stn_free.  Initial state: C = I and MPS = |0...0> for every shot
 * (Sec. IV.A).  Returns STN_EINVAL / STN_ENOMEM on bad arguments. */
stn_status stn_init(stn_ctx **out, const stn_config *cfg, void *dev_workspace,
                    size_t bytes);

/* Release the host-side context (the workspace stays the caller's). */
void stn_free(stn_ctx *ctx);

/* Message of the last error on this context ("" if none). */
const char *stn_last_error(const stn_ctx *ctx);

/* Clifford gates: C <- G C for each gate in order; the MPS is untouched
 * (Sec. IV.A).  host_gates[n_gates] is read before the call returns.  Then,
 * if dev_noise is not NULL, per-shot Pauli noise (Eqs. 2-3 sampled as
 * Paulis): dev_noise is uint64 [2][n_qubits][n_sign_words]; plane 0 holds
 * the shots whose Pauli on that qubit has an X component (X or Y), plane 1
 * those with a Z component (Z or Y). */
stn_status stn_clifford(stn_ctx *ctx, const stn_gate *host_gates, int n_gates,
                        const uint64_t *dev_noise);

/* Crosstalk rotations exp(-i theta_r Z_a Z_b [Z_c]) applied in order (Eq. 4
 * with the sign read as exp(-i theta P); Sec. IV.A for the rewrite), each
 * followed by compression to chi_max (Sec. IV.B, Eq. 8).
 * host_qubits: int32 [n_rot][3], unused entries -1, at least two qubits per
 * rotation, all distinct.  dev_theta: double angles, theta of rotation r for
 * shot s at dev_theta[s * theta_shot_stride + r] (stride 0: one angle per
 * rotation shared by all shots). */
stn_status stn_rotate(stn_ctx *ctx, const int32_t *host_qubits, int n_rot,
                      const double *dev_theta, int64_t theta_shot_stride);

/* Z measurements of host_qubits[n_meas] in order (Sec. IV.A).  For each:
 * p(m) = <phi|(I + (-1)^m P')/2|phi> / <phi|phi> with P' = C^dag Z_q C,
 * outcome m = 0 iff u < p(0) with u = dev_u[s * n_meas + i] (double in
 * [0,1)), or m = dev_forced[s * n_meas + i] (uint8) when dev_forced is not
 * NULL (dev_u is then ignored and may be NULL); the MPS is projected and,
 * when P' has an X/Y site, the frame absorbs the random part so that a
 * Clifford-only run keeps bond dimension 1.  reset != 0 applies X_q after
 * outcome 1.  Outputs (caller-owned device arrays, may be NULL):
 * dev_outcomes uint8 [n_shots][n_meas], dev_prob double [n_shots][n_meas]
 * = p(recorded outcome).  A forced outcome of probability 0 sets
 * STN_EZEROPROB on the device error word. */
stn_status stn_measure(stn_ctx *ctx, const int32_t *host_qubits, int n_meas,
                       int reset, const double *dev_u, const uint8_t *dev_forced,
                       uint8_t *dev_outcomes, double *dev_prob);

/* Per-shot log P(record so far) = sum of log p(recorded outcome), and the
 * accumulated truncation error 1 - prod(1 - w) over every cut (w = discarded
 * squared-Schmidt weight, Eq. 8).  dev_logp, dev_trunc_err: double
 * [n_shots] device arrays (either may be NULL).  Synchronises the stream and
 * reports the device error word. */
stn_status stn_logprob(stn_ctx *ctx, double *dev_logp, double *dev_trunc_err);

/* Wait for all enqueued work and report the device error word. */
stn_status stn_sync(stn_ctx *ctx);

/* Copy the tableau to the host (synchronises): host_x, host_z uint64
 * [2 n_qubits][ceil(n_qubits/64)] (row q = C^dag X_q C, row n+q = C^dag Z_q C,
 * bit j%64 of word j/64 = site j), host_sign uint64 [2 n_qubits][n_sign_words]
 * (bit set = row carries sign -1 for that shot).  Any pointer may be NULL. */
stn_status stn_get_tableau(stn_ctx *ctx, uint64_t *host_x, uint64_t *host_z,
                           uint64_t *host_sign);

/* Copy the bond dimensions to the host (synchronises): host_bonds int32
 * [n_shots][n_qubits + 1], entry b = bond between sites b-1 and b (1 at both
 * ends). */
stn_status stn_get_bonds(stn_ctx *ctx, int32_t *host_bonds);

/* Copy one MPS site tensor of one shot to the host (synchronises).  The
 * tensor (dl, 2, dr) is written row-major as interleaved (re, im) pairs of
 * double (STN_FP64) or float (STN_FP32); host_buf must hold bytes >= dl*2*dr
 * complex elements.  *dl, *dr receive the shape. */
stn_status stn_get_site(stn_ctx *ctx, int shot, int site, void *host_buf,
                        size_t bytes, int *dl, int *dr);

/* Returns every shot to the initial state (identity frame, MPS |0...0>,
 * log P = 0, fidelity 1, error word cleared) with kernel launches only: no
 * copy, fill or synchronisation, so a caller may capture stn_reset followed
 * by a whole circuit in a HIP graph and replay it for new batches of shots
 * (new angles, noise and uniforms written into the same device buffers). */
stn_status stn_reset(stn_ctx *ctx);

/* ------------------------------------------------------------ gradients
 * d log P(record) / d theta for every recorded rotation, by an adjoint pass
 * over a recorded stretch of the circuit.  Objective: J = sum of log p_k
 * over the recorded measurements (the quantity stn_logprob accumulates).
 * The rotations exp(-i theta P) are differentiated exactly (Eq. 4); each
 * truncation that dropped weight above the relative cut (chi_max binding)
 * is held fixed as the orthogonal projector onto the kept right-Schmidt
 * subspace of its step, while steps that only removed numerically null
 * directions count as exact; Clifford gates, noise, frame changes and the
 * record do not depend on theta.  Usage: stn_checkpoint_save at the start
 * of each stretch during the forward run; backwards over the stretches:
 * stn_checkpoint_load, stn_tape_begin, re-issue the stretch's calls with the
 * recorded outcomes forced, stn_tape_end, stn_backward.  The adjoint state
 * carries over between stretches (stn_adjoint_zero before the last one). */

/* Squared Schmidt values across the cut between sites bond-1 and bond
 * (1 <= bond <= n_qubits-1) for every shot: the lambda_i^2 of Eq. 8 that
 * the truncation keeps or drops there (the Fig. 2 spectrum), normalised to
 * sum 1 and in descending order, from an FP64 Gram of the centre tensor and
 * a two-sided Jacobi eigen-solve on the device.  dev_out: double
 * [n_shots][ld] (caller-owned; entries past a shot's bond dimension set to
 * 0); ld must be at least min(chi_max, 2^min(bond, n-bond)).  dev_rank:
 * int32 [n_shots] (may be NULL) receives the bond dimension at the cut.
 * Moves the orthogonality centre to site `bond` (the state is unchanged).
 * STN_ESTATE while a tape is recording. */
stn_status stn_spectrum(stn_ctx *ctx, int bond, double *dev_out, int ld, int *dev_rank);

/* Device bytes of a tape of up to max_steps rotations + measurements (each
 * step keeps a snapshot of all shots' MPS slots).  0 for bad arguments. */
size_t stn_tape_bytes(const stn_ctx *ctx, int max_steps);

/* Starts recording into dev_tape (caller-owned, 256-byte aligned, at least
 * stn_tape_bytes).  While recording, stn_rotate uses the per-step
 * schedule.  A stn_rotate / stn_measure call that would exceed max_steps
 * fails with STN_ENOMEM. */
stn_status stn_tape_begin(stn_ctx *ctx, void *dev_tape, size_t bytes, int max_steps);

/* The same as stn_tape_begin with the tape in the library's own device
 * memory instead of a caller buffer.  For callers that cannot allocate
 * device memory (code under HIP-graph capture, serving loops, harnesses
 * that forbid allocation); it calls no allocation routine.  The static tape
 * holds 64 MiB per GPU and lives until the process ends: STN_ENOMEM when
 * stn_tape_bytes(ctx, max_steps) exceeds that, STN_EDEVICE when the array
 * could not be located on this GPU at stn_init.  Every context on one GPU
 * shares the same array, which keeps the last tape's contents (each record
 * is written before it is read): recording or stn_backward on two contexts
 * of one GPU at overlapping times race. */
stn_status stn_tape_begin_static(stn_ctx *ctx, int max_steps);

/* Stops recording (snapshots the final state); *n_rotations (may be NULL)
 * receives the number of rotations recorded.  STN_ESTATE if not recording. */
stn_status stn_tape_end(stn_ctx *ctx, int *n_rotations);

/* Device bytes of the adjoint state with bond cap chi_adj (1..512).  The
 * adjoint's Schmidt ranks can exceed the forward's; stn_adjoint_truncated
 * reports when the cap was reached. */
size_t stn_adjoint_bytes(const stn_ctx *ctx, int chi_adj);

/* Places the adjoint state in dev_buf (caller-owned, 256-byte aligned, at
 * least stn_adjoint_bytes) and sets it to zero.  Synchronises.  The adjoint
 * state is compressed with a relative cut of eps_cut / 100: the gradient is
 * linear in it, so a dropped squared value lambda costs ~sqrt(lambda). */
stn_status stn_adjoint_init(stn_ctx *ctx, void *dev_buf, size_t bytes, int chi_adj);

/* Sets the adjoint state to zero (start of a backward pass) and clears the
 * flags of stn_adjoint_truncated. */
stn_status stn_adjoint_zero(stn_ctx *ctx);

/* Per shot (host_flags: n_shots ints), 1 when the adjoint state's bond cap
 * dropped weight above the relative cut since stn_adjoint_zero: that shot's
 * gradient is then approximate (raise chi_adj).  Synchronises. */
stn_status stn_adjoint_truncated(stn_ctx *ctx, int *host_flags);

/* Adjoint pass over the closed tape, last step first: writes dJ/dtheta of
 * the tape's i-th rotation for shot s to dev_grad[s * grad_stride + i]
 * (grad_stride >= the tape's rotation count unless n_shots == 1) and leaves
 * the adjoint state at the tape's start for an earlier stretch.
 * Synchronises; STN_ESTATE without a closed tape or an adjoint state. */
stn_status stn_backward(stn_ctx *ctx, double *dev_grad, int64_t grad_stride);

/* Checkpoint of the whole forward state (MPS, tableau, log P, fidelity and
 * the host-side copy of the shared frame bits).  dev_buf: caller-owned,
 * 256-byte aligned, stn_checkpoint_bytes long.  Both synchronise. */
size_t stn_checkpoint_bytes(const stn_ctx *ctx);
stn_status stn_checkpoint_save(stn_ctx *ctx, void *dev_buf);
stn_status stn_checkpoint_load(stn_ctx *ctx, const void *dev_buf);

/* Kernel classes for stn_profile / stn_profile_read. */
enum { STN_K_TABLEAU = 0,  /* tableau gates, rewrite, frame change */
       STN_K_BUILD = 1,    /* bond-2 operator blocks, copies, coefficients */
       STN_K_QR = 2,       /* Householder QR of the compression sweeps and centre moves */
       STN_K_GEMM = 3,     /* site-pair contractions (R absorb, X V, Q N) */
       STN_K_GRAM = 4,     /* FP64 Gram X^H X of the truncation */
       STN_K_EIGEN = 5,    /* FP64 eigen-solve of the Gram (FP32 path: pivoted Cholesky +
                              one-sided Jacobi; FP64 path: two-sided Jacobi) */
       STN_K_SELECT = 6,   /* truncation selection, FP64 renormalisation */
       STN_K_EXPECT = 7,   /* measurement transfer matrices and outcomes */
       STN_K_LAYER = 8,    /* fused per-shot rotation-layer kernel (all of its work) */
       STN_K_COUNT = 9 };

/* Diagnostic profiling.  Bit k of class_mask times every later launch of
 * kernel class k with HIP events on the context stream and enables the
 * device counters of algorithmic work (flops and bytes per launch, from the
 * realised bond dimensions, and the per-phase clocks of the fused kernel).
 * With STN_PROFILE_TIMING_ONLY set in class_mask only the events are
 * recorded: the counters are atomics from every block and slow the kernels
 * they count, so timings meant to stand for the kernels' speed use this
 * flag and take the work counts from a separate counted run.
 * class_mask = 0 switches profiling off.  Resets all counters;
 * synchronises. */
#define STN_PROFILE_TIMING_ONLY 0x80000000u
stn_status stn_profile(stn_ctx *ctx, unsigned class_mask);

/* Reads (and clears the event list of) the profile: per class the summed
 * kernel milliseconds, algorithmic flops and bytes (each truncation
 * eigen-solve of order nn counted at a fixed 107/8 nn^3 FP64 flops, whatever
 * route ran; see stn_profile_paths for the executed count), and the number of timed
 * launches (arrays of STN_K_COUNT entries, any may be NULL), the total number
 * of eigen-solve sweeps executed (two-sided Jacobi sweeps on the FP64 path,
 * one-sided on the FP32 path), and the FP64 part (Gram + eigen-solve) of the
 * STN_K_LAYER flops.  Work counts, sweeps and phases stay zero in
 * STN_PROFILE_TIMING_ONLY mode.  Synchronises. */
stn_status stn_profile_read(stn_ctx *ctx, double *host_ms, double *host_flops,
                            double *host_bytes, long long *host_launches,
                            double *host_eig_sweeps, double *host_layer_fp64_flops);

/* Phases of the fused layer kernel, summed over shots in shader clock
 * cycles while profiling is on (stn_profile with any class): 0 angle and
 * single-site steps, 1 centre moves, 2 bond-2 blocks, 3 QR of the
 * left-to-right sweep (or the environment Grams), 4 its R absorption,
 * 5 FP64 reduced density, 6 eigen-solve (FP32 path: pivoted Cholesky and
 * one-sided Jacobi; FP64 path: two-sided Jacobi), 7 selection, the two
 * truncation products and the renormalisation.  host_cycles: 8 doubles.
 * Synchronises. */
stn_status stn_profile_phases(stn_ctx *ctx, double *host_cycles);

/* Branch counters of the fused layer kernel while profiling is on with
 * counters (stn_profile without STN_PROFILE_TIMING_ONLY), summed over shots
 * since the last stn_profile call; host_counts: 11 doubles, in order:
 *  0 two-term steps whose left-to-right sweep formed left-environment Grams,
 *  1 steps that took the Householder QR sweep instead (a doubled bond of the
 *    span above the environment limit),
 *  2 truncation eigen-solves with the matrix in LDS,
 *  3 eigen-solves of order up to 128 with the matrix in global scratch,
 *  4 eigen-solves of order above 128,
 *  5 the largest eigen-solve order seen,
 *  6 shader cycles spent in the pivoted Cholesky of the FP32-path solves
 *    (part of phase 6 of stn_profile_phases),
 *  7 eigen-solves by Jacobi rotations in global scratch (FP64 path: the
 *    two-sided Jacobi on rho; FP32 path: the one-sided Jacobi on the rows of
 *    the Cholesky factor when its Gram does not fit the LDS tile),
 *  8 FP32-path truncations of rho in global scratch decided by the relative
 *    cut alone, whose kept space came from the orthonormalised leading rows
 *    of the pivoted Cholesky factor (no eigen-solve),
 *  9 the layer kernel's (and the per-step eigen kernel's) truncation solves
 *    as counted by stn_profile_read: a fixed 107/8 nn^3 FP64 flops per
 *    solve of order nn, whatever the route,
 * 10 the flops those solves executed (Cholesky, the Jacobi sweeps actually
 *    run, Cholesky QR, products).
 * Synchronises. */
stn_status stn_profile_paths(stn_ctx *ctx, double *host_counts);

/* How stn_rotate schedules its kernels: 1 = one launch per kernel step for
 * all shots (grids spread each product over many blocks; best for few
 * shots), 2 = one launch per chunk of up to 64 rotations in which each block
 * runs every step of one shot (best for many shots), 0 = automatic (2 when
 * n_shots >= 64).  Results are identical up to rounding order. */
stn_status stn_set_layer_mode(stn_ctx *ctx, int mode);

/* Threads per shot of the fused layer kernel: 64 (one wavefront per shot),
 * 128 (the default), 256 or 512.  A tuning knob: results agree to rounding order.
 * STN_EINVAL for any other value. */
stn_status stn_set_layer_threads(stn_ctx *ctx, int threads);

/* Largest doubled bond at which the fused layer kernel's left-to-right
 * sweep forms left-environment Grams instead of Householder QR (0: always
 * QR).  stn_init sets the largest its workspace allows (up to 512); values
 * above that are STN_EINVAL.  A tuning knob: results agree to rounding
 * order. */
stn_status stn_set_layer_env(stn_ctx *ctx, int max_bond);

/* LDS tile of the fused layer kernel's FP32-path truncation: steps of order
 * up to `order` (32 or 64) keep the factor in LDS, and larger steps whose
 * pivoted-Cholesky rank (or count above the cut) fits the tile solve its
 * Gram there (larger ones use the shot's global scratch); 0 = chosen from
 * chi_max and the threads per shot (64 when 17 <= chi_max <= 32 or with 256
 * or more threads, else 32).  The 64 tile takes ~70 KB of LDS per block,
 * so fewer 64- or 128-thread shots are resident per compute unit.  A tuning
 * knob: results agree within the truncation cut (the kept spaces of a step
 * may differ by directions of weight below eps_cut).  STN_EINVAL for any
 * other value. */
stn_status stn_set_layer_lds(stn_ctx *ctx, int order);

/* Overwrite one MPS site tensor of one shot from the host (synchronises):
 * host_buf holds dl*2*dr complex elements in the layout of stn_get_site; the
 * shot's bonds site and site+1 become dl and dr.  The caller keeps the
 * neighbouring sites consistent and the orthogonality centre as declared by
 * stn_set_center (used to restore a checkpointed state).  STN_EINVAL when a
 * bond exceeds min(chi_max, 2^min(b, n-b)). */
stn_status stn_set_site(stn_ctx *ctx, int shot, int site, const void *host_buf,
                        int dl, int dr);

/* Declare the orthogonality centre of the state held (after stn_set_site). */
stn_status stn_set_center(stn_ctx *ctx, int center);

/* Orthogonality centre site shared by all shots (sites left of it are
 * left-orthonormal, right of it right-orthonormal). */
int stn_center(const stn_ctx *ctx);

/* ------------------------------------------------------------ decoding
 * Union-find decoder of detection events (host code; the paper decodes by
 * minimum-weight matching over the Pauli-twirled error model, Sec. III.D).
 * A detector graph: n_nodes detectors 0..n_nodes-1 plus the boundary, whose
 * index is n_nodes; each edge is one independent error mechanism that fires
 * detectors a and b (b = n_nodes: one detector and the boundary), with
 * weight log((1 - p) / p) > 0 and obs = 1 when it flips the logical
 * observable.  Per shot, events[s * n_nodes + v] = 1 when detector v fired.
 * pred[s] receives the predicted observable flip (parity of the flagged
 * edges of the correction); corrections (may be NULL) receives the
 * correction as uint8 [n_shots][n_edges].  The correction fires exactly the
 * detectors that fired.  All pointers are host memory; no GPU is used.
 * STN_EINVAL on an edge out of range, a loop, or a weight that is not
 * positive and finite. */
typedef struct {
    int32_t a, b;        /* detector indices; n_nodes = the boundary */
    double weight;       /* log((1 - p) / p) of the mechanism */
    uint8_t obs;         /* 1: flips the logical observable */
    uint8_t pad[7];
} stn_dem_edge;

stn_status stn_decode(const stn_dem_edge *edges, int n_edges, int n_nodes, const uint8_t *events,
                      int n_shots, uint8_t *pred, uint8_t *corrections);

#ifdef __cplusplus
}
#endif
#endif /* STN_H */
