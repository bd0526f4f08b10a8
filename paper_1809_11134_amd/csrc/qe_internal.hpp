// Internal interface between the libqe host code and its kernel translation
// units (launchers run on the caller's stream and return hipError_t).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qe {

struct BatchArgs {
    int32_t B;
    int32_t uniform_n;
    const int8_t* nq;
    int32_t uniform_L;
    const int32_t* goff;
    const uint16_t* gates;
    int64_t num_gates;
    int64_t tstride;
    const int64_t* toff;
    const void* targets;
    int64_t num_telems;
    int32_t mode;           // QE_FIT_*
    int32_t mix_w5;         // wavefronts per width-5 circuit in the sorted mixed launch (1 or 2)
    const uint32_t* angles; // per-gate angles (u32 turn fractions, parallel to gates) or null
    uint32_t* err;          // device error word (atomicOr of QE_DEVERR_*)
};

// api.hip: schedule of the FP32 path for circuits of width n and length L:
// LDS-staged (lds = 1) or register-resident kernel, the LDS kernels'
// wavefronts per circuit, circuits per workgroup of the one-wavefront
// population kernels
struct Sched {
    int lds, waves, cpb;
};
// Library class of a schedule (QE_SCHED_*): circuits as given in a discrete
// library, circuits the QEQEA sampler decodes (only {I, NOT, CNOT, CV, CV+}:
// the CV body), circuits with angled gates (Ising library).
enum : int { SCHED_DISCRETE = 0, SCHED_SAMPLED = 1, SCHED_ISING = 2, SCHED_CLASSES = 3 };
Sched schedule_for(int n, int L, int lib_class = SCHED_DISCRETE);
// MFMA paths: the fewest non-identity gates a group needs to be fused into a
// block (smaller groups go gate by gate in FP32), per width and length class
int mfma_min_block(int n, int L);
bool schedule_lds(int n);

// Workspace of a mixed-width batch: MIX_WORK_META int32 of item table, then
// the B circuit indices in cost order.
constexpr int MIX_WORK_META = 32;

// eval.hip
// work: MIX_WORK_META + B int32 of device workspace for mixed-width batches
// (order of circuits by width and length); NULL selects one filtered launch
// per width.
hipError_t launch_eval_fp32(const BatchArgs& a, int path, float* f, float* g, float* delta,
                            int32_t* work, hipStream_t s);
// Phase-insensitive mode only (a no-op otherwise): marks circuits whose
// target has an entry of modulus strictly between 0 and 1 (NaN outputs,
// QE_DEVERR_TARGET); launched after the evaluation.
hipError_t launch_target_check(const BatchArgs& a, bool fp64, void* f, void* g, void* delta,
                               hipStream_t s);
// The two halves of the sorted mixed-width launch: the cost order of the
// batch's circuits into work (it depends only on widths and lengths), and
// the evaluation of a batch in an order computed before.
hipError_t launch_mix_sort(const BatchArgs& a, int32_t* work, hipStream_t s);
hipError_t launch_mix_eval(const BatchArgs& a, const int32_t* work, float* f, float* g, float* delta,
                           hipStream_t s);
hipError_t launch_eval_lds(const BatchArgs& a, bool fp64, void* f, void* g, void* delta,
                           hipStream_t s);
hipError_t launch_unitary(const BatchArgs& a, bool fp64, void* out, hipStream_t s);

// dense.hip: every gate expanded to its full segment matrix and multiplied
// (the paper's steps 3-5; an ablation baseline, any widths, angles allowed)
hipError_t launch_eval_dense(const BatchArgs& a, float* f, float* g, float* delta, hipStream_t s);

// mfma.hip: fused 4-wire gate blocks on MFMA (uniform width 5 or 6)
hipError_t launch_eval_mfma(const BatchArgs& a, bool fp16, bool renorm, float* f, float* g,
                            float* delta, hipStream_t s);

// Encoding state of one slot (Eq. 10 index), 16 bytes (eight to a 128-byte
// line): every field the loop reads or writes for a slot lies in one line,
// so a random slot access costs one line.  `key` is the slot's segment
// fitness in the current generation (Sec. IV-E.1: the largest fitness of the
// circuits that used it), as the bits of that non-negative float plus one
// (so unsigned order is float order), 0 = unused.  Any circuit whose fitness
// equals it may apply the slot's elitism: the update is the same for all of
// them, so repeats leave the same state.
struct SlotRec {
    uint32_t theta;        // qubit angle as a turn fraction (2^32 = 2 pi)
    uint32_t best_theta;   // state of the best segment fitness seen
    float best_f;          // best segment fitness seen, -1 = never used
    uint32_t key;
};
static_assert(sizeof(SlotRec) == 16, "slot records are 16 bytes");

// Workgroups are dispatched round-robin over the eight XCDs, each with its
// own L2: block j of a range of n blocks that starts at a multiple of 8 is
// the (j / 8)-th block to reach XCD j % 8.  The returned index gives every
// XCD one contiguous share of the range, taken in order, so that the
// circuits of one population (whose slot records share lines) run under
// one L2.
__device__ __forceinline__ uint32_t xcd_swizzle(uint32_t j, uint32_t n) {
    const uint32_t q = n >> 3, r = n & 7u, x = j & 7u;
    return x * q + (x < r ? x : r) + (j >> 3);
}

__device__ __forceinline__ uint32_t seg_key(float f) { return __float_as_uint(f) + 1u; }
__device__ __forceinline__ float seg_fitness(uint32_t key) { return __uint_as_float(key - 1u); }

// Qutrit of a rotation slot (s < n*L*P) and its best copy, one 64-byte line.
struct QutritRec {
    float q[6];            // three complex amplitudes (re, im)
    float bq[6];
    float pad[4];
};

// Encoding-state arguments of the QEQEA / GA loop kernels.
struct LoopArgs {
    int32_t n, lib, L, P, I;
    int32_t fit_mode;                  // QE_FIT_*
    uint64_t seed;
    uint64_t thr_pm, thr_pc, thr_pg;   // probability thresholds, floor(p * 2^32)
    float r32;                         // mutation step per unit (1 - segFit), in 2^-32 turns
    uint32_t R;                        // regions of Eq. 10 (rotations, then templates)
    uint32_t S;                        // slots per instance: R*L*P
    uint32_t Q;                        // qutrits per instance: n*L*P
    SlotRec* slot;                     // [I][S]
    QutritRec* qrec;                   // [I][Q]
    uint16_t* genomes[2];              // GA double buffer
    const float* target32;             // [I][N][N] complex64
    const double* target64;            // [I][N][N] complex128
    // Mutation decisions as bitmaps, double-buffered by generation parity:
    // generation g sets bit ind of mask g & 1 for every individual that
    // mutates and clears mask (g + 1) & 1, which generation g - 1 consumed.
    // The host clears both before a generation that does not follow the
    // previous one.
    uint32_t* mutmask;                 // [2][I][MW]
    uint32_t MW;                       // words per instance: ceil(P / 32)
    float* inst_best_f;                // per instance
    uint16_t* inst_best_gates;         // [I][L] (L = the longest genome of a mixed GA)
    uint32_t* inst_best_angles;        // [I][L] (Ising library; zero otherwise)
    const float* su3_tab;              // [4][4096]: cos/sin of angles, cos/sin of phases
    const uint64_t* gen_ptr;           // device generation base (graphs) or null
    uint32_t* err;
    // Mixed GA populations (null otherwise): population i has inst_n[i]
    // wires and genomes of inst_L[i] genes; its P genomes start at gene
    // inst_goff[i] of each genome buffer, its target at complex element
    // inst_toff[i] of the target buffers.  n and L then hold the maxima.
    const int32_t* inst_n;
    const int32_t* inst_L;
    const int64_t* inst_goff;
    const int64_t* inst_toff;
    int64_t genes;                     // genes per genome buffer (all populations)
    // QEQEA, populations of at most DEDUP_MAX_ENTRIES entries (P * L) of at
    // most 256 positions and fewer than 2^31 slots: per (circuit, position)
    // entry of a generation, its slot index, with bit 31 set if another
    // circuit uses the same slot; two buffers of I * P * L words, generation g
    // in buffer g & 1, so that the search of the next generation can run
    // while the current one's words are read (null otherwise)
    uint32_t* dup;
    // with dup: per generation parity and population, the entries whose slot
    // is shared ({entry index within the population, slot}, [2][I][P * L])
    // and their number ([2][I])
    uint2* shared_list;
    uint32_t* shared_count;
};
constexpr uint32_t DUP_SHARED = 0x80000000u;
constexpr int DEDUP_MAX_ENTRIES = 4096;
// words of the search's LDS hash table for a population of `entries`
// entries: at most half full, whole multiples of 256 (at most 32 KB)
__host__ __device__ inline uint32_t dedup_table(uint32_t entries) { return (2u * entries + 255u) & ~255u; }

// loop.hip
hipError_t launch_qeqea_init(const LoopArgs& a, hipStream_t s);
hipError_t launch_ga_init(const LoopArgs& a, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// angles: the circuits' gate angles [I*P*L] (written for the Ising library,
// read by the evaluation and the update), null for the discrete libraries.
hipError_t launch_qeqea_sample(const LoopArgs& a, uint64_t gen, uint32_t* slots, uint16_t* gates,
                               uint32_t* angles, hipStream_t s);
hipError_t launch_ga_copy(const LoopArgs& a, uint64_t gen, uint16_t* gates, hipStream_t s);
hipError_t launch_eval_population(const LoopArgs& a, const uint16_t* gates, const uint32_t* angles,
                                  float* f, hipStream_t s);
hipError_t launch_qeqea_fused(const LoopArgs& a, uint64_t gen, uint32_t* slots, uint16_t* gates,
                              uint32_t* angles, float* f, bool decide, hipStream_t s);
hipError_t launch_mutation_decisions(const LoopArgs& a, uint64_t gen, hipStream_t s);
hipError_t launch_scatter(const LoopArgs& a, uint64_t gen, const uint32_t* slots, const float* f,
                          hipStream_t s);
// slots: the generation's slot indices [I*P*L], or NULL to draw them again
// from the SAMPLE stream (the internal generation path).
// shared: the generation was sampled by the fused kernel after the
// shared-slot search, so its slot words say which slots the fused kernel
// committed (false: every entry's slot goes through the keys).
// dedup_next: the same launch runs the shared-slot search of generation
// gen + 1 (needs a.dup).
hipError_t launch_qeqea_update(const LoopArgs& a, uint64_t gen, const uint32_t* slots,
                               const uint16_t* gates, const uint32_t* angles, const float* f,
                               hipStream_t s, bool shared = false, bool dedup_next = false);
// the slot words of generation gen (buffer gen & 1 of a.dup), before its
// fused kernel
hipError_t launch_dedup(const LoopArgs& a, uint64_t gen, hipStream_t s);
hipError_t launch_mutmask_clear(const LoopArgs& a, hipStream_t s);
// Dense copy of one field of the encoding state (which: 0 theta, 1 qutrit
// amplitudes, 2 best_f, 3 best_theta, 4 best qutrit amplitudes).
hipError_t launch_state_gather(const LoopArgs& a, int which, void* dst, hipStream_t s);
hipError_t launch_ga_eval(const LoopArgs& a, uint64_t gen, float* f, hipStream_t s);
hipError_t launch_ga_update(const LoopArgs& a, uint64_t gen, const float* f, hipStream_t s);
hipError_t launch_c128_to_c64(const double* src, float* dst, int64_t n_reals, hipStream_t s);
hipError_t launch_gen_advance(uint64_t* gen_ptr, uint64_t by, hipStream_t s);
hipError_t launch_gen_set(uint64_t* gen_ptr, uint64_t v, hipStream_t s);
// cand: elite_cand_keys(I, P) 64-bit keys of device workspace.
size_t elite_cand_keys(int I, int P);
hipError_t launch_elite_select(const LoopArgs& a, const float* f, int k, int32_t* idx,
                               unsigned long long* cand, hipStream_t s);
hipError_t launch_elite_eval(const LoopArgs& a, const uint16_t* gates, const uint32_t* angles, int k,
                             const int32_t* idx, double* f64, hipStream_t s);

}  // namespace qe
