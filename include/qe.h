/*
 * qe.h -- C ABI of libqe, an MI355X (gfx950) implementation of the hot path of
 * the Quantum Encoded Quantum Evolutionary Algorithm (QEQEA) and its classical
 * GA baseline (Krylov & Lukac, arXiv:1809.11134): batched fitness evaluation
 * of candidate circuits (Sec. IV-E, Eq. 11), circuit construction by sampling
 * the qubit/qutrit encoding (Sec. IV-D, Eq. 10), segment fitness, elitism and
 * adaptive mutation (Secs. IV-E.1, IV-F, Eq. 12), and the GA operators of
 * Sec. V-B, for discrete gate libraries and for the Ising gate model of
 * Sec. III (Eqs. 3-6).
 *
 * Conventions shared by every entry point
 *  - Gate descriptor (uint16): kind in bits 0-3, target wire in bits 4-7,
 *    control wire in bits 8-11, bits 12-15 zero.  Kinds: 0 I, 1 NOT, 2 CNOT,
 *    3 CV, 4 CV+ (V = sqrt(NOT)), 5 H, 6 T.  Single-qubit kinds ignore the
 *    control field.
 *  - Ising kinds (Sec. III): 7 R_x, 8 R_y, 9 R_z (Eqs. 3-5) on the target
 *    wire, 10 the interaction J (Eq. 6, read with the exponent i theta:
 *    exp(-i theta/2 Z_a Z_b), a diagonal of e^{-+i theta/2}) on the wires
 *    a = target field, b = control field (a != b).  Each carries an angle:
 *    a uint32 fraction of a full turn, theta = 2 pi u / 2^32, in an array
 *    parallel to the descriptors ("angles"); without one these kinds are
 *    invalid descriptors.
 *  - Wire w of an n-wire register is bit (n-1-w) of a basis-state index: the
 *    first Kronecker factor is the most significant (Eqs. 1-2).
 *  - A circuit g_0 .. g_{L-1} denotes U = G_{L-1} ... G_0 (g_0 acts first).
 *  - Matrices are row-major; complex64 = interleaved (re, im) float pairs,
 *    complex128 = interleaved double pairs.
 *  - Fitness (Eq. 11): f = 1 - sqrt((2^n - |tr(U^dagger T)|) / 2^n), computed
 *    through the identity 2^n - |tr(T^dagger U)| = (1/2)||U T^dagger -
 *    e^{i arg tr} I||_F^2 so that single precision keeps its accuracy near
 *    f = 1; the radicand is clamped to [0, 1].  g = |tr(T^dagger U)| / 2^n
 *    and delta = 2^n - |tr| are optional outputs.
 *  - Pointers named *_dev are device memory owned by the caller (the library
 *    never frees them); *_host are host memory.  All calls taking `stream`
 *    (a hipStream_t passed as void*, NULL = the null stream) are asynchronous:
 *    they validate host-side arguments, enqueue kernels and return without
 *    synchronising.  Calls documented as "syncs" block on `stream`.
 *  - Errors: every call returns a qe_status.  Invalid host arguments return
 *    QE_ERR_INVALID (nothing is enqueued).  Malformed device-side data
 *    (descriptors, widths, offsets out of range) cannot be checked before the
 *    launch: the kernels never access memory out of bounds for it, write NaN
 *    for the affected circuit and raise a device error flag that
 *    qe_device_errors() reports.  qe_last_error() gives a message for the
 *    last failing call of the calling thread.
 *  - A context is not thread-safe; use it from one host thread and one
 *    stream at a time.
 */
#ifndef QE_H
#define QE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qe_status;
enum {
    QE_OK = 0,
    QE_ERR_INVALID = 1,     /* bad argument; nothing was launched */
    QE_ERR_UNSUPPORTED = 2, /* valid but not implemented (e.g. QEQEA on library 1) */
    QE_ERR_DEVICE = 3,      /* a HIP call failed */
    QE_ERR_OOM = 4,         /* device allocation failed */
    QE_ERR_NUMERIC = 5,     /* NaN/Inf met (qe_get_best) */
    QE_ERR_STATE = 6        /* call out of order (e.g. no targets set) */
};

enum { QE_LIB_NCV = 0,      /* {I, NOT, CNOT, CV, CV+} */
       QE_LIB_HT_NCV = 1,   /* {H, T, CNOT, CV, CV+}   */
       QE_LIB_ISING = 2 };  /* {R_x, R_y, R_z, J} with angles (QEQEA only) */
enum { QE_ALG_QEQEA = 0, QE_ALG_GA = 1 };
enum { QE_PATH_FP32 = 0,        /* per-gate row updates, FP32, tuned schedule per width */
       QE_PATH_FP32_REG = 1,    /* forced: matrix held in registers, one wave per circuit */
       QE_PATH_FP32_LDS = 2,    /* forced: matrix staged in LDS, columns split over waves */
       QE_PATH_MFMA_BF16 = 3,   /* fused 4-wire gate blocks on MFMA, bf16 hi+lo, FP32
                                   accumulation, columns renormalised after each block */
       QE_PATH_MFMA_FP16 = 4,   /* same with fp16 hi+lo (lo scaled by 2^11) */
       QE_PATH_MFMA_BF16_RAW = 5,  /* bf16 hi+lo without renormalisation */
       QE_PATH_MFMA_FP16_RAW = 6,  /* fp16 hi+lo without renormalisation */
       QE_PATH_DENSE = 7 };        /* ablation: the paper's segment matrices (Sec. IV-C,
                                      steps 3-5), every gate expanded by Kronecker products
                                      to 2^n x 2^n and multiplied densely, FP32, any widths */

/* Device error flags (bitmask) raised by kernels. */
enum { QE_DEVERR_DESC = 1,      /* invalid gate descriptor */
       QE_DEVERR_WIDTH = 2,     /* circuit width outside 1..6 */
       QE_DEVERR_RANGE = 4,     /* gate, target or mutation-list index outside its buffer */
       QE_DEVERR_NUMERIC = 8,   /* NaN/Inf fitness */
       QE_DEVERR_TARGET = 16 }; /* phase-insensitive fitness of a target with an
                                   entry of modulus strictly between 0 and 1 */

/* ------------------------------------------------------------------ batches */
/* A batch of circuits to evaluate (Sec. IV-E).  Host struct; the arrays it
 * points to live on the device.
 *   num_circuits   B >= 0.
 *   uniform_n      > 0: every circuit has this many wires (1..6) and n_qubits
 *                  may be NULL; 0: widths from n_qubits[B] (int8).
 *   uniform_L      > 0: circuit b is gates[b*uniform_L .. +uniform_L) and
 *                  gate_offsets may be NULL; 0: gates[gate_offsets[b] ..
 *                  gate_offsets[b+1]) with gate_offsets[B+1] (int32).
 *   num_gates      number of descriptors in `gates` (bounds for offsets).
 *   target_stride  >= 0: target b at targets + b*target_stride complex
 *                  elements (0 = one shared target); < 0: at
 *                  targets + target_offsets[b] (int64, complex elements).
 *   targets        complex64 (FP32/MFMA paths) or complex128 (FP64 calls),
 *                  2^n x 2^n row-major per target.
 *   num_target_elems  complex elements in `targets` (bounds).
 *   fitness_mode   QE_FIT_EQ11 (0) or QE_FIT_PHASE_INSENSITIVE (1).
 *   angles_dev     NULL (discrete gates only), or one uint32 angle per entry
 *                  of gates_dev (same indexing), read for the Ising kinds.
 *                  Angled batches run on QE_PATH_FP32 / QE_PATH_FP32_LDS /
 *                  QE_PATH_DENSE and the FP64 calls; the register and MFMA
 *                  paths return QE_ERR_UNSUPPORTED for them.
 *
 * Fitness modes.  QE_FIT_EQ11: Eq. 11 as printed, f = 1 - sqrt((2^n -
 * |tr(T^dagger U)|) / 2^n), computed through the exact identity 2^n - |tr| =
 * 1/2 ||U T^dagger - e^{i arg tr} I||_F^2 (g = |tr| / 2^n, delta = 2^n - |tr|).
 * QE_FIT_PHASE_INSENSITIVE: f = 1 - sqrt(r) with r = sum_{i != j}
 * |(U T^dagger)_ij|^2 / 2^n, clamped to [0, 1] (g = 1 - r, delta = 2^n r).
 * For a unitary U, 1 - r = sum_i |(U T^dagger)_ii|^2 / 2^n, which for a
 * permutation target T (the paper's targets) equals sum_ij |U_ij|^2
 * |T_ij|^2 / 2^n, the phase-insensitive reading of Eq. 11 under which the
 * paper's Table II figure reproduces; it ignores the global phase and
 * phases applied after the circuit.  The two agree exactly when every entry
 * of T has modulus 0 or 1 (a permutation with phases, as the paper's targets
 * are); the evaluation calls check each target in this mode and give a
 * circuit whose target has an entry of modulus strictly between 0 and 1 (by
 * more than 1e-5, FP64 calls 1e-9) f = g = delta = NaN and QE_DEVERR_TARGET. */
enum { QE_FIT_EQ11 = 0, QE_FIT_PHASE_INSENSITIVE = 1 };

typedef struct {
    int32_t num_circuits;
    int32_t uniform_n;
    const int8_t* n_qubits_dev;
    int32_t uniform_L;
    const int32_t* gate_offsets_dev;
    const uint16_t* gates_dev;
    int64_t num_gates;
    int64_t target_stride;
    const int64_t* target_offsets_dev;
    const void* targets_dev;
    int64_t num_target_elems;
    int32_t fitness_mode;
    const uint32_t* angles_dev;
} qe_batch;

/* Fitness of every circuit of the batch against its target, Eq. 11 of
 * Sec. IV-E (the hot path; batch->fitness_mode selects the phase-insensitive
 * mode).  path: QE_PATH_*.  f_dev [B] required; g_dev,
 * delta_dev [B] optional (NULL).  The 2^n x 2^n product U T^dagger is built
 * gate by gate from T^dagger (FP32 paths), block by block (MFMA paths:
 * uniform width 5 or 6 only, QE_ERR_UNSUPPORTED otherwise) or segment matrix
 * by segment matrix (QE_PATH_DENSE, the paper's scheme, N^3 work per gate).  Circuits whose
 * width, gates or target are malformed get f = NaN (see qe_device_errors).
 * ctx may be NULL. */
typedef struct qe_ctx qe_ctx;
qe_status qe_eval_fitness(qe_ctx* ctx, const qe_batch* batch, int32_t path, float* f_dev,
                          float* g_dev, float* delta_dev, void* stream);
/* How a mixed-width batch (uniform_n == 0) runs on QE_PATH_FP32: with a
 * workspace, in one launch whose workgroups take the circuits in cost order
 * (widest first, then longest first), the order computed on the device into
 * the workspace; without one, in one launch per width.  Both give the same
 * results.  qe_eval_fitness uses the workspace of ctx when ctx is a context
 * of mixed populations (qe_create_mixed) and the batch fits it (calls on one
 * context must then not overlap); it allocates nothing and never
 * synchronises. */

/* Bytes of device workspace qe_eval_fitness_ws needs for num_circuits
 * circuits (0 for num_circuits < 0). */
size_t qe_eval_workspace_bytes(int32_t num_circuits);

/* qe_eval_fitness with a caller-owned device workspace of workspace_bytes
 * bytes (at least qe_eval_workspace_bytes(batch->num_circuits), else
 * QE_ERR_INVALID), used by mixed-width batches on QE_PATH_FP32 and ignored
 * otherwise.  Calls sharing a workspace must not overlap. */
qe_status qe_eval_fitness_ws(const qe_batch* batch, int32_t path, float* f_dev, float* g_dev,
                             float* delta_dev, void* workspace_dev, size_t workspace_bytes,
                             void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * qe_eval_fitness_ws without a workspace argument.  The workspace is a
 * fixed device array inside the library, one per GPU, held until the
 * process ends (4 * (32 + QE_NOALLOC_MAX_CIRCUITS) bytes); the call
 * allocates nothing and frees nothing.  A mixed-width batch of more than
 * QE_NOALLOC_MAX_CIRCUITS circuits on QE_PATH_FP32 returns QE_ERR_INVALID
 * (nothing is launched).  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  Results equal qe_eval_fitness_ws. */
#define QE_NOALLOC_MAX_CIRCUITS 262144
qe_status qe_eval_fitness_noalloc(const qe_batch* batch, int32_t path, float* f_dev, float* g_dev,
                                  float* delta_dev, void* stream);

/* The same fitness in FP64 (targets complex128), for re-checking elite
 * circuits; f_dev required, g_dev/delta_dev optional. */
qe_status qe_eval_fitness_fp64(const qe_batch* batch, double* f_dev, double* g_dev,
                               double* delta_dev, void* stream);

/* The unitary U = G_{L-1}...G_0 of every circuit (Eqs. 1-6 with the library
 * gates), written to out_dev as [B][2^n][2^n] complex64 (precision 0) or
 * complex128 (precision 1).  Requires batch->uniform_n > 0; out_elems is the
 * capacity of out_dev in complex elements; targets are ignored. */
qe_status qe_build_unitary(const qe_batch* batch, int32_t precision, void* out_dev,
                           int64_t out_elems, void* stream);

/* Reads and clears the device error flags raised since the last call
 * (QE_DEVERR_* bitmask) on the current device.  Syncs the device. */
qe_status qe_device_errors(int32_t* flags_host);

/* ---------------------------------------------------------------- contexts */
/* Parameters of the evolutionary search (Sec. IV-B, IV-F, V-B):
 *   n_qubits (numberOfWires) 2..6 for QEQEA, 1..6 for GA; library QE_LIB_*;
 *   algorithm QE_ALG_*; size_of_individual L (circuit length) 1..1024;
 *   size_of_population P (circuits per instance per generation) 1..65536
 *   (QEQEA 1..16384, GA 1..4096);
 *   n_instances I independent populations, each with its own target;
 *   prob_mutation (probabilityOfMutation, QEQEA) in [0, 1];
 *   mutation_range (mutationRange, radians) in [0, 2 pi);
 *   ga_crossover_prob, ga_gene_mutation_prob in [0, 1] (GA);
 *   seed: the Philox4x32-10 key;
 *   fitness_mode: QE_FIT_* (the fitness the search maximises; see qe_batch).
 * QEQEA decodes to the library {I, NOT, CNOT, CV, CV+} or to the Ising
 * library; the GA takes the discrete libraries only (its genome holds no
 * angles). */
typedef struct {
    int32_t n_qubits;
    int32_t library;
    int32_t algorithm;
    int32_t size_of_individual;
    int32_t size_of_population;
    int32_t n_instances;
    float prob_mutation;
    float mutation_range;
    float ga_crossover_prob;
    float ga_gene_mutation_prob;
    uint64_t seed;
    int32_t fitness_mode;
} qe_problem;

/* Creates a context on the current device: allocates the ctx-owned encoding
 * (QEQEA: R * L * P slot records of 16 bytes (angle, best angle, best
 * segment fitness, the generation's segment key), R = n + n(n-1) regions for
 * {I, NOT, CNOT, CV, CV+} (one template per ordered wire pair) or
 * n + n(n-1)/2 for the Ising library (one per unordered pair), and n*L*P
 * qutrit records of 64 bytes (3 complex64 amplitudes and their best copy);
 * GA: two L*P genome buffers) per instance,
 * and initialises it as the population initialisation of Sec. IV-B (angles
 * from the Philox INIT stream, qutrits (1,1,1)/sqrt(3), no best yet).  Syncs. */
qe_status qe_create(const qe_problem* problem, qe_ctx** ctx_out);
qe_status qe_destroy(qe_ctx* ctx);

/* A GA search (Sec. V-B) over I = problem->n_instances independent
 * populations of P circuits each, population i on n_qubits_host[i] wires
 * (1..6) with genomes of lengths_host[i] genes (1..1024): the uneven batches
 * of circuits built in parallel (Sec. IV-D) evaluated in one launch per
 * generation, the circuits taken in cost order (widest, then longest first;
 * the order is fixed by the widths and lengths and computed here once).
 * problem->algorithm must be QE_ALG_GA, library QE_LIB_NCV or QE_LIB_HT_NCV;
 * problem->n_qubits and size_of_individual are ignored and stored as the
 * largest width and length.  Genomes of population i are drawn from the
 * INIT stream with instance index i over the library of its own width, as
 * a context of that width alone would draw them.  Targets
 * (qe_set_targets) are packed: population i's 2^n_i x 2^n_i matrix follows
 * those of populations 0..i-1.  Every call taking a context accepts a mixed
 * one, with these layouts: circuits of population i (qe_sample,
 * qe_eval_population, qe_update, qe_elite_recheck gates) start at gene
 * P * (L_0 + ... + L_{i-1}), circuit k of it at that plus k * L_i; fitness
 * arrays stay [I][P]; qe_get_best returns L_i gates.  Syncs. */
qe_status qe_create_mixed(const qe_problem* problem, const int32_t* n_qubits_host,
                          const int32_t* lengths_host, qe_ctx** ctx_out);

/* Copies the I targets ([I][2^n][2^n] complex128, device) into the context
 * (kept in complex128 for the FP64 re-check and in complex64 for the hot
 * path).  Must precede sample/eval/update/generation.  Asynchronous, except
 * for a context whose fitness_mode is QE_FIT_PHASE_INSENSITIVE: then it
 * checks every target (modulus 0 or 1 entries, see qe_batch), syncs, and
 * returns QE_ERR_UNSUPPORTED (targets not taken) if one fails. */
qe_status qe_set_targets(qe_ctx* ctx, const void* targets_c128_dev, void* stream);

/* Circuit construction (Sec. IV-D).  QEQEA: for each instance i, circuit
 * k < P and position pos < L, draws whichIndividual and
 * whichRotationOrInteraction from the Philox SAMPLE stream of generation
 * `gen`, forms the segment index of Eq. 10 into slots_dev[(i*P+k)*L + pos]
 * and decodes that segment into gates_dev[(i*P+k)*L + pos]: the qutrit of a
 * rotation slot is measured by the Born rule; for the Ising library the
 * gate is the rotation about the measured axis (or J on the template's
 * pair) and takes the slot's angle (written to angles_dev, required then);
 * for {I, NOT, CNOT, CV, CV+} the angle is rounded to quarter turns
 * (angles_dev ignored, may be NULL).  GA: copies the current population
 * (slots_dev may be NULL). */
qe_status qe_sample(qe_ctx* ctx, uint64_t gen, uint32_t* slots_dev, uint16_t* gates_dev,
                    uint32_t* angles_dev, void* stream);

/* Fitness of the I*P circuits in gates_dev (with angles_dev for the Ising
 * library, NULL otherwise) against each instance's target (FP32 path);
 * f_dev [I*P]. */
qe_status qe_eval_population(qe_ctx* ctx, const uint16_t* gates_dev, const uint32_t* angles_dev,
                             float* f_dev, void* stream);

/* One update step (Secs. IV-E.1, IV-F; GA: Sec. V-B).  QEQEA: every slot used
 * in generation `gen` takes the largest fitness of the circuits it built;
 * a used slot that beats its recorded best stores its state, otherwise
 * reverts to it; each individual mutates with prob_mutation (all qubits by
 * +-(1 - segFit) * mutation_range, or all qutrits by one SU(3) step of
 * Eq. 12, equiprobably).  GA: SUS selection, two-point crossover, gene
 * mutation, best individual kept.  slots_dev/gates_dev/angles_dev/f_dev as
 * produced by qe_sample and qe_eval_population for the same `gen`
 * (angles_dev: Ising library only, NULL otherwise).  QEQEA with slots_dev
 * NULL: allowed only right after qe_sample_eval(gen) on this context (else
 * QE_ERR_STATE); the segment keys and decisions that call left are used,
 * with the slot indices of its shared-slot search (the update then handles
 * only the slots several circuits shared, and runs the next generation's
 * search) or, for populations too large for the search, drawn again from
 * the SAMPLE stream. */
qe_status qe_update(qe_ctx* ctx, uint64_t gen, const uint32_t* slots_dev,
                    const uint16_t* gates_dev, const uint32_t* angles_dev, const float* f_dev,
                    void* stream);

/* sample + eval + update of generation `gen` (QEQEA: the fused kernel and
 * the update, preceded by the shared-slot search described at
 * qe_sample_eval unless the update of generation gen - 1 on this context
 * already ran it; GA: two launches); f_dev [I*P] receives the generation's
 * fitness (may be NULL).  Results equal qe_sample, qe_eval_population and
 * qe_update in sequence. */
qe_status qe_generation(qe_ctx* ctx, uint64_t gen, float* f_dev, void* stream);

/* The first half of qe_generation for QEQEA (the launches qe_generation and
 * qe_run_graph make before the update): circuit construction (as qe_sample,
 * into gates_dev, and into slots_dev unless it is NULL) fused with the
 * fitness evaluation (f_dev), the segment fitness (Sec. IV-E.1) and the
 * generation's mutation decisions (Sec. IV-F).  For populations of at most
 * 4096 (circuit, position) entries and 256 positions, a search for the slots
 * that more than one circuit uses runs first (skipped when the context holds
 * its result already: the slots drawn depend on the seed and the generation
 * only, and the update after qe_sample_eval, qe_generation and every
 * generation of qe_run_graph searches the next generation's slots; the
 * context keeps the results of two generations, so calls on one context
 * must be ordered, one stream or synchronised), and the fused kernel commits
 * the elitism of every slot its circuit alone used (its segment fitness is
 * that circuit's fitness, final as soon as the circuit is evaluated); the
 * shared slots keep the largest fitness for qe_update.  The encoding is then
 * partly updated: sampling generation gen again (qe_sample) sees the
 * committed states, so sample it before.  qe_update(gen, slots, gates,
 * angles, f) afterwards completes the generation with the same result as
 * qe_generation (with slots_dev it runs the elitism of every slot, which
 * leaves a committed slot as it is); with slots_dev NULL there, it is the
 * last launch of qe_generation alone.  angles_dev as in qe_sample.  QEQEA
 * only. */
qe_status qe_sample_eval(qe_ctx* ctx, uint64_t gen, uint32_t* slots_dev, uint16_t* gates_dev,
                         uint32_t* angles_dev, float* f_dev, void* stream);

/* Captures and instantiates the graph that qe_run_graph(n_gen, f_hist_dev)
 * replays, without running it (so that a later qe_run_graph does no capture
 * work).  Syncs nothing; safe to call again (no-op when cached). */
qe_status qe_graph_prepare(qe_ctx* ctx, int32_t n_gen, float* f_hist_dev);

/* Runs generations first_gen .. first_gen + n_gen - 1 as one HIP graph
 * (captured on first use for this n_gen and f_hist_dev, then replayed);
 * f_hist_dev [n_gen][I*P] or NULL.  Same results as n_gen qe_generation
 * calls. */
qe_status qe_run_graph(qe_ctx* ctx, uint64_t first_gen, int32_t n_gen, float* f_hist_dev,
                       void* stream);

/* FP64 re-check of elite circuits: for each instance, the k circuits of
 * gates_dev with the highest f_dev (ties: lowest index) are re-evaluated in
 * FP64 against the complex128 target.  gates_dev NULL: the circuits of the
 * last generation run by qe_generation / qe_run_graph (f_dev must then be
 * that generation's fitness; angles_dev is ignored).  angles_dev: the
 * circuits' angles (Ising library, required with gates_dev), NULL
 * otherwise.  idx_dev [I][k] (int32, circuit index within the instance),
 * f64_dev [I][k].  1 <= k <= P <= 4096.  The selection uses a workspace the
 * context owns, so re-checks on one context must not overlap (one stream). */
qe_status qe_elite_recheck(qe_ctx* ctx, const uint16_t* gates_dev, const uint32_t* angles_dev,
                           const float* f_dev, int32_t k, int32_t* idx_dev, double* f64_dev,
                           void* stream);

/* Best circuit seen so far by instance `instance` (over every generation run
 * through qe_update / qe_generation / qe_run_graph): its L gates, their
 * angles (Ising library; zeros otherwise), its FP32 fitness and its FP64
 * re-evaluated fitness.  Any output may be NULL.  Syncs the device. */
qe_status qe_get_best(qe_ctx* ctx, int32_t instance, uint16_t* gates_host, uint32_t* angles_host,
                      float* f32_host, double* f64_host);

/* Checkpoint / restore of the whole encoding state (bit-exact; the run is a
 * pure function of the state, the seed and the generation index).  With
 * buf_host NULL, qe_checkpoint stores the needed size in *size.  Both sync. */
qe_status qe_checkpoint(qe_ctx* ctx, void* buf_host, size_t* size);
qe_status qe_restore(qe_ctx* ctx, const void* buf_host, size_t size);

/* Dense copy of one field of the context-owned state, for tests and
 * inspection (the QEQEA state is stored per slot as one record, so each field
 * is gathered).  which: 0 theta (u32, [I][S] slot order of Eq. 10), 1 qutrit
 * amplitudes (f32, 6 per qutrit, [I][n*L*P]), 2 best_f (f32), 3 best_theta
 * (u32), 4 best qutrit amplitudes (f32), 5 GA genomes of generation parity 0
 * (u16, [I][P][L]), 6 parity 1, 7 QEQEA mutation decisions (u32 bitmaps
 * [2][I][ceil(P/32)]: bit ind of map g & 1 is set when individual ind
 * mutates in generation g).  *elems receives the field's size in
 * elements (0 when the algorithm has no such field); with dst_dev non-NULL
 * (device memory of that size, caller-owned) the copy is enqueued on
 * `stream`.  Unknown which: QE_ERR_INVALID. */
qe_status qe_state_read(qe_ctx* ctx, int32_t which, void* dst_dev, int64_t* elems, void* stream);

/* Gate-library table used by the GA (instance index -> descriptor), host
 * output of qe_lib_size() entries; discrete libraries only (qe_lib_size
 * returns -1 and qe_lib_table QE_ERR_INVALID for the others). */
int32_t qe_lib_size(int32_t library, int32_t n_qubits);
qe_status qe_lib_table(int32_t library, int32_t n_qubits, uint16_t* table_host);

/* Schedule of the QE_PATH_FP32 path: for width n (1..6), lds != 0 selects
 * the LDS-staged kernel, 0 the register-resident one (n <= 3 always use the
 * one-element-per-lane kernel).  Process-wide; the defaults come from the
 * tuning table measured on MI355X and can be overridden by the environment
 * variable QE_SCHEDULE="n:lds,n:lds,...". */
qe_status qe_set_schedule(int32_t n_qubits, int32_t lds);
qe_status qe_get_schedule(int32_t n_qubits, int32_t* lds);

/* The whole schedule of width n for circuits of length class lclass (0: L <
 * 32, 1: L >= 32; batches of uneven lengths use class 1): lds as above,
 * waves = wavefronts per circuit of the LDS-staged kernels (1 for n <= 4, 1
 * or 2 for n = 5, 4 for n = 6), cpb = circuits per workgroup of the
 * one-wavefront population kernels (1 or 4).  Process-wide, like
 * qe_set_schedule; the tuning table (lines "n lclass lds waves cpb") and
 * QE_SCHEDULE="n:lds[:waves[:cpb]],..." set it too.  Every LDS-staged
 * schedule gives the same results bit for bit (the fitness reduction runs
 * in an order fixed by the width); the register-resident kernel agrees
 * within the FP32 tolerance.  A mixed-population context keeps the width-5
 * wave count it was created with.  Unknown combinations: QE_ERR_INVALID. */
qe_status qe_set_schedule_ex(int32_t n_qubits, int32_t lclass, int32_t lds, int32_t waves, int32_t cpb);
qe_status qe_get_schedule_ex(int32_t n_qubits, int32_t lclass, int32_t* lds, int32_t* waves, int32_t* cpb);

/* Library classes of the schedule table: the best kernel shape depends on
 * what the gates are.  QE_SCHED_DISCRETE: circuits given in a discrete
 * library (qe_eval_fitness, qe_eval_population, the GA); QE_SCHED_SAMPLED:
 * circuits the QEQEA sampler decodes from the encoding of Sec. IV-D (only
 * I, NOT, CNOT, CV, CV+: qe_sample_eval and the generation kernels);
 * QE_SCHED_ISING: circuits of the Ising library (Sec. III), whose gates
 * carry angles (batches with angles_dev, Ising contexts).  Angled circuits
 * of 4 or more wires always take the LDS-staged kernels, whatever lds says. */
enum { QE_SCHED_DISCRETE = 0, QE_SCHED_SAMPLED = 1, QE_SCHED_ISING = 2 };

/* The schedule of one (width, length class, library class).
 * qe_set_schedule_ex sets all three library classes at once and
 * qe_get_schedule_ex reads the QE_SCHED_DISCRETE one; tuning table lines
 * "n lclass lib lds waves cpb" set one class, the shorter forms all of them.
 * Arguments and errors as for qe_set_schedule_ex, plus lib_class 0..2. */
qe_status qe_set_schedule_lib(int32_t n_qubits, int32_t lclass, int32_t lib_class, int32_t lds,
                              int32_t waves, int32_t cpb);
qe_status qe_get_schedule_lib(int32_t n_qubits, int32_t lclass, int32_t lib_class, int32_t* lds,
                              int32_t* waves, int32_t* cpb);

/* MFMA paths (QE_PATH_MFMA_*): consecutive gates within four wires are fused
 * into a 16 x 16 block applied on the matrix cores; a group of fewer than
 * min_block non-identity gates is applied gate by gate in FP32 instead (the
 * block's construction and its three hi/lo products cost more than a few
 * row-pair updates).  min_block 1 fuses every group; 65 never fuses (a group
 * holds at most the 64 gates of a descriptor chunk).  Per width and length
 * class (lclass as above), process-wide; tuning table lines
 * "mfma n lclass min_block".  The results stay within the MFMA paths'
 * stated error (the FP32 gate updates are the more accurate part).
 * QE_ERR_INVALID for a width outside 1..6, lclass not 0/1, min_block
 * outside 1..65 or a NULL output. */
qe_status qe_set_mfma_min_block(int32_t n_qubits, int32_t lclass, int32_t min_block);
qe_status qe_get_mfma_min_block(int32_t n_qubits, int32_t lclass, int32_t* min_block);

/* Measurement helper (not part of the method): the LDS bandwidth the GPU
 * sustains, the denominator of the per-gate kernels' LDS rooflines.  Launches
 * `workgroups` workgroups of 256 threads, each owning 32 KB of LDS, whose
 * threads run `iters` iterations of eight conflict-free 16-byte LDS accesses
 * (every wavefront instruction moves one contiguous kilobyte).  mode 0:
 * reads (ds_read_b128); 1: writes (ds_write_b128); 2: a read and a write of
 * each word (a copy within LDS).  sink_dev: caller-owned device memory of
 * workgroups * 256 uint32 (written, so no access can be optimised away).
 * *bytes_host (may be NULL) receives the LDS bytes the launch moves (reads
 * plus writes).  Asynchronous on `stream`; time it with events. */
qe_status qe_probe_lds(int32_t mode, int32_t workgroups, int32_t iters, uint32_t* sink_dev,
                       double* bytes_host, void* stream);

/* Measurement helper (not part of the method): the rate of random 16-byte
 * record accesses in HBM, the floor of the QEQEA update (whose slot records
 * are 16 bytes, one 128-byte line per random access).  Launches `accesses`
 * threads; thread t takes record h(t) mod count of records_dev (count
 * 16-byte records of caller-owned device memory; h a hash of t and salt,
 * uniform over the buffer), reads it (mode 0) or reads it and writes it back
 * changed (mode 1).  sink_dev: one caller-owned uint32, written only for a
 * record pattern the caller's buffer does not hold.  count and accesses up
 * to 2^32 - 1.  Asynchronous on `stream`; time it with events.
 * QE_ERR_INVALID for a bad mode, NULL pointers or sizes out of range. */
qe_status qe_probe_records(int32_t mode, void* records_dev, int64_t count, int64_t accesses, uint32_t salt,
                           uint32_t* sink_dev, void* stream);

const char* qe_last_error(void);
const char* qe_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QE_H */
