// The cheap loop around the fitness evaluation: circuit construction by
// sampling the encoding (Sec. IV-D), segment fitness / elitism / adaptive
// mutation (Secs. IV-E.1, IV-F), the GA operators of Sec. V-B, population
// initialisation (Sec. IV-B) and the FP64 re-check of elite circuits.
//
// Everything that decides an integer or updates the encoding is written one
// rounding per operation so that it is reproducible bit for bit: the library
// is compiled with -ffp-contract=off (no multiply-add fusion anywhere) and the
// pragma below repeats that for this file.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "../../include/qe.h"
#include "qe_eval_core.hpp"
#include "qe_internal.hpp"

#pragma clang fp contract(off)

namespace qe {

__device__ __forceinline__ uint32_t gen_of(const LoopArgs& a, uint64_t gen) {
    return (uint32_t)(a.gen_ptr ? *a.gen_ptr + gen : gen);
}

// The slot words of generation gen (buffer gen & 1 of the shared-slot search's
// output).
__device__ __forceinline__ uint32_t* dup_words(const LoopArgs& a, uint32_t gen) {
    return a.dup + (size_t)(gen & 1u) * ((size_t)a.I * a.P * a.L);
}

// ------------------------------------------------------------- measurement
// Born-rule measurement of a qutrit (3 complex amplitudes, unnormalised):
// u in [0,1) from the top 24 bits of w scales the cumulative weights.
__device__ __forceinline__ int measure_amps(float2 a0, float2 a1, float2 a2, uint32_t w) {
    const float p0 = a0.x * a0.x + a0.y * a0.y;
    const float p1 = a1.x * a1.x + a1.y * a1.y;
    const float p2 = a2.x * a2.x + a2.y * a2.y;
    const float c0 = p0, c1 = c0 + p1, c2 = c1 + p2;
    const float u = (float)(w >> 8) * 0x1p-24f;
    const float x = u * c2;
    return x < c0 ? 0 : (x < c1 ? 1 : 2);
}

// An empty instruction sequence that reads v: the value must exist at this
// point, so the compiler can neither drop the work that produces it nor sink
// that work into a later branch.
__device__ __forceinline__ void anchor(float v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void anchor(uint32_t v) { asm volatile("" ::"v"(v)); }

// The state a slot's decode reads: its angle and, for a rotation slot, its
// qutrit amplitudes.  Both loads are issued by every lane before either
// value is used (a template slot reads qutrit 0 of its instance, one cached
// line, and ignores it), so the gather costs one random-access latency, not
// two in sequence.
struct SlotState {
    uint32_t theta;
    float2 q0, q1, q2;
};

struct QState {
    float q[6], bq[6];
};

__device__ __forceinline__ QState load_qstate(const QutritRec* r) {
    const float4* p = reinterpret_cast<const float4*>(r);
    const float4 x = p[0], y = p[1], z = p[2];
    return QState{{x.x, x.y, x.z, x.w, y.x, y.y}, {y.z, y.w, z.x, z.y, z.z, z.w}};
}

__device__ __forceinline__ void store_qstate(QutritRec* r, const QState& s) {
    float4* p = reinterpret_cast<float4*>(r);
    p[0] = make_float4(s.q[0], s.q[1], s.q[2], s.q[3]);
    p[1] = make_float4(s.q[4], s.q[5], s.bq[0], s.bq[1]);
    p[2] = make_float4(s.bq[2], s.bq[3], s.bq[4], s.bq[5]);
}

__device__ __forceinline__ SlotState load_slot_state(const LoopArgs& a, uint32_t i, uint32_t s, bool rot) {
    SlotState st;
    st.theta = a.slot[(size_t)i * a.S + s].theta;
    const float2* q = reinterpret_cast<const float2*>(a.qrec[(size_t)i * a.Q + (rot ? s : 0u)].q);
    st.q0 = q[0];
    st.q1 = q[1];
    st.q2 = q[2];
    return st;
}

// A slot's whole record and (rotation slot) qutrit record, as the fused
// kernel gathers them for the first 64 positions: decoding needs the angle
// and the qutrit, and a slot no other circuit uses is committed from them.
struct SlotFull {
    SlotRec r;
    QState q;
};

__device__ __forceinline__ SlotFull load_slot_full(const LoopArgs& a, uint32_t i, uint32_t s, bool rot) {
    SlotFull f;
    f.r = a.slot[(size_t)i * a.S + s];
    f.q = load_qstate(a.qrec + (size_t)i * a.Q + (rot ? s : 0u));
    return f;
}

__device__ __forceinline__ SlotState state_of(const SlotFull& f) {
    SlotState st;
    st.theta = f.r.theta;
    st.q0 = make_float2(f.q.q[0], f.q.q[1]);
    st.q1 = make_float2(f.q.q[2], f.q.q[3]);
    st.q2 = make_float2(f.q.q[4], f.q.q[5]);
    return st;
}

// Decodes slot s of instance i: rotation slot -> NOT on its wire when the
// measured axis is x and the angle rounds to a half turn, else I; template
// slot (c, t) -> controlled V^q with q the angle in quarter turns.
// (FULL: the whole records are loaded and returned in *full)
template <bool FULL = false>
__device__ __forceinline__ uint16_t decode_slot(const LoopArgs& a, uint32_t gen, uint32_t i,
                                                uint32_t s, SlotFull* full = nullptr) {
    const uint32_t LP = (uint32_t)a.L * (uint32_t)a.P;
    const uint32_t r = s / LP;
    const bool rot = r < (uint32_t)a.n;
    SlotState st;
    if constexpr (FULL) {
        *full = load_slot_full(a, i, s, rot);
        st = state_of(*full);
    } else {
        st = load_slot_state(a, i, s, rot);
    }
    // every lane measures (a wavefront with any rotation slot runs the draw
    // anyway) while the loads are in flight; template slots ignore the outcome
    const u32x4 w = draw(a.seed, TAG_MEASURE, gen, i, s);
    anchor(w.x);
    anchor(st.q0.x);
    anchor(st.q2.x);
    const int axis = measure_amps(st.q0, st.q1, st.q2, w.x);
    const int q = (int)(((st.theta + 0x20000000u) >> 30) & 3u);
    if (rot) return (axis == 0 && q == 2) ? make_desc(KIND_NOT, (int)r, 0) : (uint16_t)0;
    if (q == 0) return 0;
    int c, t;
    pair_of(a.n, (int)r - a.n, &c, &t);
    const int kind = q == 1 ? KIND_CV : (q == 2 ? KIND_CNOT : KIND_CVDG);
    return make_desc(kind, t, c);
}

// Ising library (Secs. IV-A, IV-C): a rotation slot on wire w becomes the
// rotation about the measured axis (outcome 0, 1, 2 = x, y, z) on w, a
// template slot on the unordered pair (a, b) the interaction J on (a, b);
// both take the slot's angle.  Returns {descriptor, angle}.
template <bool FULL = false>
__device__ __forceinline__ uint2 decode_ising(const LoopArgs& a, uint32_t gen, uint32_t i, uint32_t s,
                                              SlotFull* full = nullptr) {
    const uint32_t LP = (uint32_t)a.L * (uint32_t)a.P;
    const uint32_t r = s / LP;
    const bool rot = r < (uint32_t)a.n;
    SlotState st;
    if constexpr (FULL) {
        *full = load_slot_full(a, i, s, rot);
        st = state_of(*full);
    } else {
        st = load_slot_state(a, i, s, rot);
    }
    const u32x4 w = draw(a.seed, TAG_MEASURE, gen, i, s);   // every lane, as in decode_slot
    anchor(w.x);
    anchor(st.q0.x);
    anchor(st.q2.x);
    const int axis = measure_amps(st.q0, st.q1, st.q2, w.x);
    if (rot) return make_uint2(make_desc(KIND_RX + axis, (int)r, 0), st.theta);
    int pa, pb;
    upair_of(a.n, (int)r - a.n, &pa, &pb);
    return make_uint2(make_desc(KIND_ZZ, pa, pb), st.theta);
}

// Segment index of Eq. 10 from the SAMPLE draw of position pos: the
// individual and the region are drawn, the position is the circuit's own.
__device__ __forceinline__ uint32_t slot_of_draw(const LoopArgs& a, const u32x4& w, uint32_t pos) {
    const uint32_t ind = scale_u32(w.x, (uint32_t)a.P);
    const uint32_t region = scale_u32(w.y, a.R);
    return region * (uint32_t)a.L * (uint32_t)a.P + ind * (uint32_t)a.L + pos;
}

// Segment index for circuit k, position pos of instance i.
__device__ __forceinline__ uint32_t sample_slot(const LoopArgs& a, uint32_t gen, uint32_t i,
                                                uint32_t k, uint32_t pos) {
    return slot_of_draw(a, draw(a.seed, TAG_SAMPLE, gen, i, k * (uint32_t)a.L + pos), pos);
}

// --------------------------------------------------------------------- init
__global__ void qeqea_init_kernel(LoopArgs a, float amp) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)a.I * a.S;
    if (idx >= total) return;
    const uint32_t i = (uint32_t)(idx / a.S), s = (uint32_t)(idx % a.S);
    const u32x4 w = draw(a.seed, TAG_INIT, GEN_INIT, i, s);
    SlotRec r;
    r.theta = w.x;
    r.best_theta = w.x;
    r.best_f = -1.0f;
    r.key = 0u;
    a.slot[idx] = r;
    if (s < a.Q) {
        QutritRec q;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            q.q[c] = (c & 1) ? 0.0f : amp;
            q.bq[c] = q.q[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) q.pad[c] = 0.0f;
        a.qrec[(size_t)i * a.Q + s] = q;
    }
}

__global__ void ga_init_kernel(LoopArgs a) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)a.P * a.L;
    if (idx >= (size_t)a.I * per) return;
    const uint32_t i = (uint32_t)(idx / per), item = (uint32_t)(idx % per);
    const u32x4 w = draw(a.seed, TAG_INIT, GEN_INIT, i, item);
    a.genomes[0][idx] = lib_desc(a.lib, a.n, (int)scale_u32(w.x, (uint32_t)lib_size(a.lib, a.n)));
}

// Mixed populations: workgroup i draws the P x inst_L[i] genes of population
// i over the library of its own width.
__global__ void ga_init_mixed_kernel(LoopArgs a) {
    const uint32_t i = blockIdx.x;
    const int n = a.inst_n[i];
    const uint32_t per = (uint32_t)a.P * (uint32_t)a.inst_L[i], nl = (uint32_t)lib_size(a.lib, n);
    uint16_t* g = a.genomes[0] + a.inst_goff[i];
    for (uint32_t item = threadIdx.x; item < per; item += blockDim.x) {
        const u32x4 w = draw(a.seed, TAG_INIT, GEN_INIT, i, item);
        g[item] = lib_desc(a.lib, n, (int)scale_u32(w.x, nl));
    }
}

__global__ void inst_best_init_kernel(LoopArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.I) return;
    a.inst_best_f[i] = -1.0f;
    if (a.mutmask)
        for (uint32_t w = 0; w < 2 * a.MW; ++w)
            a.mutmask[((size_t)(w / a.MW) * a.I + i) * a.MW + w % a.MW] = 0u;
    for (int l = 0; l < a.L; ++l) {
        a.inst_best_gates[(size_t)i * a.L + l] = 0;
        a.inst_best_angles[(size_t)i * a.L + l] = 0u;
    }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) p[idx] = v;
}

__global__ void gen_advance_kernel(uint64_t* g, uint64_t by) { *g += by; }
__global__ void gen_set_kernel(uint64_t* g, uint64_t v) { *g = v; }

// ---------------------------------------------------------------- sampling
__global__ void qeqea_sample_kernel(LoopArgs a, uint64_t gen64, uint32_t* __restrict__ slots,
                                    uint16_t* __restrict__ gates, uint32_t* __restrict__ angles) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)a.P * a.L;
    if (idx >= (size_t)a.I * per) return;
    const uint32_t gen = gen_of(a, gen64);
    const uint32_t i = (uint32_t)(idx / per), rem = (uint32_t)(idx % per);
    const uint32_t k = rem / a.L, pos = rem % a.L;
    const uint32_t s = sample_slot(a, gen, i, k, pos);
    slots[idx] = s;
    if (a.lib == LIB_ISING) {
        const uint2 g = decode_ising(a, gen, i, s);
        gates[idx] = (uint16_t)g.x;
        if (angles) angles[idx] = g.y;
    } else {
        gates[idx] = decode_slot(a, gen, i, s);
    }
}

__global__ void ga_copy_kernel(LoopArgs a, uint64_t gen64, uint16_t* __restrict__ gates) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)a.genes) return;
    gates[idx] = a.genomes[gen_of(a, gen64) & 1][idx];
}

// Mutation decision of an individual for this generation (Sec. IV-F: with
// probability pm; qubit or qutrit mode equiprobably), from its MUT_IND draw.
__device__ __forceinline__ bool mutates(const LoopArgs& a, uint32_t gen, uint32_t i, uint32_t ind,
                                        bool* qutrit_mode = nullptr) {
    const u32x4 w = draw(a.seed, TAG_MUT_IND, gen, i, ind);
    if (qutrit_mode) *qutrit_mode = (w.y & 1u) != 0;
    return (uint64_t)w.x < a.thr_pm;
}

__device__ __forceinline__ uint32_t* mask_of(const LoopArgs& a, uint32_t gen, uint32_t i) {
    return a.mutmask + ((size_t)(gen & 1u) * a.I + i) * a.MW;
}

// Records that individual ind mutates in generation gen.
__device__ __forceinline__ void mark_mutation(const LoopArgs& a, uint32_t gen, uint32_t i, uint32_t ind) {
    atomicOr(mask_of(a, gen, i) + (ind >> 5), 1u << (ind & 31u));
}

// Individual ind's share of emptying the mask of the other parity.
__device__ __forceinline__ void clear_next_mask(const LoopArgs& a, uint32_t gen, uint32_t i, uint32_t ind) {
    if ((ind & 31u) == 0) mask_of(a, gen + 1u, i)[ind >> 5] = 0u;
}

// Elitism of a slot that one circuit alone used (defined with the update).
__device__ void commit_alone(const LoopArgs& a, uint32_t i, uint32_t s, float v, SlotFull f);

// -------------------------------------------- population evaluation (FP32)
// One circuit per wavefront (register / per-lane layouts, and the LDS layout
// with W = 1) or per workgroup (LDS layout, W > 1); the target is the
// circuit's instance target.  With SAMPLE the circuit is first constructed
// from the encoding (qe_sample) and afterwards every slot it used keeps the
// largest fitness of the circuits that used it (its segment key).  With
// `decide` (the internal generation) circuit k also draws the mutation
// decision of individual k (both run over 0..P-1) and empties its part of the
// decision mask of the other generation parity.
// ISING: circuits of the Ising library, whose gates carry angles (read from
// angles_in, or with SAMPLE decoded and written to angles_out).  With W > 1
// and SAMPLE only the first wavefront samples; the others take its
// descriptors from xch (two buffers of 64 entries, by chunk parity, so one
// barrier per chunk separates a chunk's writes from the next chunk's).
template <int NQ, int W, bool SAMPLE, bool ISING>
__device__ __forceinline__ void eval_circuit(const LoopArgs& a, uint32_t gen, uint32_t ci,
                                             const uint16_t* gates_in, const uint32_t* angles_in,
                                             uint32_t* slots_out, uint16_t* gates_out,
                                             uint32_t* angles_out, float* f_out, bool writer,
                                             bool decide, float2* M, uint4* gt, float (*red)[3],
                                             void* xch = nullptr) {
    const uint32_t i = ci / (uint32_t)a.P, k = ci % (uint32_t)a.P;
    const int lane = (int)lane_id();
    const int L = a.L;
    const float* T = a.target32 + (size_t)2 * i * ((size_t)1 << (2 * NQ));
    if (SAMPLE && decide && writer && lane == 0) clear_next_mask(a, gen, i, k);
    constexpr int KEEP = 4;                 // chunks of 64 slots kept for the scatter
    uint32_t kept[KEEP];
    bool alone[KEEP];                       // no other circuit of the generation uses the slot
#pragma unroll
    for (int c = 0; c < KEEP; ++c) { kept[c] = 0xFFFFFFFFu; alone[c] = false; }
    // (the flags exist only for sampled generations whose duplicates were
    // found beforehand, and then L <= KEEP * 64)
    auto is_alone = [&](uint32_t word) -> bool { return a.dup && !(word & DUP_SHARED); };
    SlotFull full0{};                       // the records of the lane's slot in chunk 0
    using SrcT = std::conditional_t<ISING, uint2, uint32_t>;
    auto own = [&](int ch) -> SrcT {
        const int p = ch * 64 + lane;
        if constexpr (!SAMPLE) {
            if constexpr (ISING)
                return p < L ? make_uint2((uint32_t)gates_in[(size_t)ci * L + p], angles_in[(size_t)ci * L + p])
                             : make_uint2(0u, 0u);
            else
                return p < L ? (uint32_t)gates_in[(size_t)ci * L + p] : 0u;
        }
        const bool pos = p < L;
        const bool dec = decide && writer && p == L;
        if (!pos && !dec) return SrcT{};
        // one Philox pass: position lanes draw their entry's individual and
        // region (or, after the shared-slot search, read the slot it drew),
        // lane L the mutation decision of individual k
        uint32_t word = 0u;
        if (a.dup && pos) {
            word = dup_words(a, gen)[(size_t)ci * L + p];
        } else {
            const u32x4 w = draw(a.seed, pos ? (uint32_t)TAG_SAMPLE : (uint32_t)TAG_MUT_IND, gen, i,
                                 pos ? k * (uint32_t)L + (uint32_t)p : k);
            if (!pos) {
                if ((uint64_t)w.x < a.thr_pm) mark_mutation(a, gen, i, k);
                return SrcT{};
            }
            word = slot_of_draw(a, w, (uint32_t)p);
        }
        const uint32_t s = a.dup ? (word & ~DUP_SHARED) : word;
        const bool al = is_alone(word);
#pragma unroll
        for (int c = 0; c < KEEP; ++c)
            if (c == ch) { kept[c] = s; alone[c] = al; }
        if constexpr (ISING) {
            // (whole records only where the fused kernel may commit them)
            const uint2 g = (ch == 0 && a.dup) ? decode_ising<true>(a, gen, i, s, &full0)
                                               : decode_ising(a, gen, i, s);
            if (writer) {
                if (slots_out) slots_out[(size_t)ci * L + p] = s;
                gates_out[(size_t)ci * L + p] = (uint16_t)g.x;
                angles_out[(size_t)ci * L + p] = g.y;
            }
            return g;
        } else {
            const uint16_t d = (ch == 0 && a.dup) ? decode_slot<true>(a, gen, i, s, &full0)
                                                  : decode_slot(a, gen, i, s);
            if (writer) {
                if (slots_out) slots_out[(size_t)ci * L + p] = s;
                gates_out[(size_t)ci * L + p] = d;
            }
            return (uint32_t)d;
        }
    };
    // the circuit's descriptors, chunk ch (every wavefront of the circuit
    // calls this the same number of times: the chunk loop is uniform)
    auto src = [&](int ch) -> SrcT {
        if constexpr (SAMPLE && W > 1) {
            SrcT* buf = reinterpret_cast<SrcT*>(xch) + (ch & 1) * 64;
            const bool first = threadIdx.x < 64;
            SrcT d{};
            if (first) {
                d = own(ch);
                buf[lane] = d;
            }
            __syncthreads();
            return first ? d : buf[lane];
        } else {
            return own(ch);
        }
    };
    float fv;
    bool ok;
    if constexpr (W == 0) {
        FitOut o;
        ok = run_width<NQ, false>(NQ, T, L, src, nullptr, &o, a.fit_mode);
        fv = o.f;
    } else {
        float gd, dd;
        RowMap map{};
        // circuits the sampler decodes hold only {I, NOT, CNOT, CV, CV+}
        constexpr bool NCV = SAMPLE && !ISING;
        ok = run_lds_path<NQ, W, false, NCV>(M, gt, T, L, src, &map, W == 1 ? 0 : -1);
        constexpr int WR = reduction_waves<NQ>();
        static_assert(WR == 1 || WR == W, "the reduction's wavefronts are the circuit's");
        if constexpr (W > 1) __syncthreads();     // every wavefront's columns are in place
        if (WR > 1)
            fv = canonical_fitness<NQ, WR>(M, map, a.fit_mode, &gd, &dd, (int)(threadIdx.x >> 6) % W, red);
        else
            fv = writer ? canonical_fitness<NQ, 1>(M, map, a.fit_mode, &gd, &dd) : 0.0f;
    }
    if (!ok) fv = __builtin_nanf("");
    if (writer && lane == 0) {
        f_out[ci] = fv;
        if (!ok) atomicOr(a.err, (uint32_t)QE_DEVERR_DESC);
        else if (!(fv == fv)) atomicOr(a.err, (uint32_t)QE_DEVERR_NUMERIC);
    }
    // segment fitness: a slot no other circuit of the generation uses takes
    // this circuit's fitness as its segment fitness and its elitism now
    // (nothing else reads or writes it before the update); every other slot
    // keeps the largest key, for the update's elitism
    if (SAMPLE && writer && fv >= 0.0f) {
        const uint32_t key = seg_key(fv);
#pragma unroll
        for (int c = 0; c < KEEP; ++c) {
            const int p = c * 64 + lane;
            if (p >= L) continue;
            if (alone[c]) {
                if (c == 0) commit_alone(a, i, kept[0], fv, full0);
                else commit_alone(a, i, kept[c], fv, load_slot_full(a, i, kept[c], kept[c] < a.Q));
            }
            else atomicMax(&a.slot[(size_t)i * a.S + kept[c]].key, key);
        }
        for (int p = KEEP * 64 + lane; p < L; p += 64) {
            const uint32_t s = sample_slot(a, gen, i, k, (uint32_t)p);
            atomicMax(&a.slot[(size_t)i * a.S + s].key, key);
        }
    }
    // a circuit length that fills whole wavefronts leaves no spare lane
    if (SAMPLE && decide && writer && (L & 63) == 0 && lane == 0 && mutates(a, gen, i, k))
        mark_mutation(a, gen, i, k);
}

template <int NQ, int W, bool SAMPLE, bool ISING = false, int CPB = (W == 1 ? 4 : 1)>
__global__ __launch_bounds__(256) void population_kernel(LoopArgs a, uint64_t gen64,
                                                         const uint16_t* __restrict__ gates_in,
                                                         const uint32_t* __restrict__ angles_in,
                                                         uint32_t* __restrict__ slots_out,
                                                         uint16_t* __restrict__ gates_out,
                                                         uint32_t* __restrict__ angles_out,
                                                         float* __restrict__ f_out, bool decide) {
    const uint32_t gen = gen_of(a, gen64);
    const uint32_t total = (uint32_t)a.I * (uint32_t)a.P;
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    if constexpr (W == 0) {
        static_assert(!ISING || NQ <= 3, "Ising circuits of 4 or more wires take the LDS-staged path");
        const uint32_t ci = __builtin_amdgcn_readfirstlane(bid * 4 + (threadIdx.x >> 6));
        if (ci >= total) return;
        eval_circuit<NQ, 0, SAMPLE, ISING>(a, gen, ci, gates_in, angles_in, slots_out, gates_out,
                                           angles_out, f_out, true, decide, nullptr, nullptr, nullptr);
    } else {
        // W = 1: CPB circuits per workgroup, one per wavefront (no barrier
        // is shared, so a wavefront past the end may leave); W > 1: one
        // circuit per workgroup of W wavefronts
        static_assert(W == 1 || CPB == 1, "one circuit per workgroup of several wavefronts");
        constexpr int N = 1 << NQ;
        __shared__ __align__(16) float2 M[CPB][N * N];
        __shared__ uint4 GT[W == 1 ? CPB : W][ISING ? GATE_TABLE_ANGLED : GATE_TABLE];
        __shared__ float red[4][3];
        const int wave = (int)(threadIdx.x >> 6);
        const uint32_t ci = W == 1 ? bid * CPB + (uint32_t)wave : bid;
        if (ci >= total) return;
        // (W > 1: the gate tables are unused, the first one is the
        // descriptor exchange)
        eval_circuit<NQ, W, SAMPLE, ISING>(a, gen, ci, gates_in, angles_in, slots_out, gates_out,
                                           angles_out, f_out, W == 1 || threadIdx.x < 64, decide,
                                           M[W == 1 ? wave : 0], GT[wave], red,
                                           W == 1 ? nullptr : static_cast<void*>(GT[0]));
    }
}

// -------------------------------------------------------------- scatter-max
// Segment fitness for the step-by-step path (qe_update): every entry raises
// its slot's key to its circuit's fitness.
__global__ void scatter_kernel(LoopArgs a, const uint32_t* __restrict__ slots,
                               const float* __restrict__ f) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)a.P * a.L;
    if (idx >= (size_t)a.I * per) return;
    const uint32_t i = (uint32_t)(idx / per);
    const float fv = f[idx / a.L];
    const uint32_t s = slots[idx];
    if (!(fv >= 0.0f) || s >= a.S) return;
    atomicMax(&a.slot[(size_t)i * a.S + s].key, seg_key(fv));
}

// Mutation decisions for the step-by-step path (qe_update): one thread per
// individual.
__global__ void mutation_decision_kernel(LoopArgs a, uint64_t gen64) {
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (uint32_t)a.I * (uint32_t)a.P) return;
    const uint32_t gen = gen_of(a, gen64), i = id / (uint32_t)a.P, ind = id % (uint32_t)a.P;
    clear_next_mask(a, gen, i, ind);
    if (mutates(a, gen, i, ind)) mark_mutation(a, gen, i, ind);
}

__global__ void mutmask_clear_kernel(LoopArgs a) {
    const size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w < (size_t)2 * a.I * a.MW) a.mutmask[w] = 0u;
}

// ------------------------------------------------------------------- update
// One SU(3) step (Eq. 12 with parameter j alone, value a*domain/4096).
__device__ __forceinline__ void su3_step(float* q, int j, int ai, const float* tab) {
    const float x0 = q[0], y0 = q[1], x1 = q[2], y1 = q[3], x2 = q[4], y2 = q[5];
    if (j <= 2) {
        const float c = tab[ai], s = tab[SU3_TAB + ai];
        if (j == 0) {          // [[c, s, 0], [-s, c, 0], [0, 0, 1]]
            q[0] = c * x0 + s * x1; q[1] = c * y0 + s * y1;
            q[2] = c * x1 - s * x0; q[3] = c * y1 - s * y0;
        } else if (j == 1) {   // [[c, 0, s], [0, 1, 0], [-s, 0, c]]
            q[0] = c * x0 + s * x2; q[1] = c * y0 + s * y2;
            q[4] = c * x2 - s * x0; q[5] = c * y2 - s * y0;
        } else {               // [[1, 0, 0], [0, c, -s], [0, s, c]]
            q[2] = c * x1 - s * x2; q[3] = c * y1 - s * y2;
            q[4] = s * x1 + c * x2; q[5] = s * y1 + c * y2;
        }
    } else if (j <= 4) {
        const float c = tab[2 * SU3_TAB + ai], s = tab[3 * SU3_TAB + ai];
        if (j == 3) {          // q0 *= e^{i phi}
            q[0] = c * x0 - s * y0; q[1] = s * x0 + c * y0;
        } else {               // q1 *= e^{i phi}
            q[2] = c * x1 - s * y1; q[3] = s * x1 + c * y1;
        }
        q[4] = c * x2 + s * y2; q[5] = c * y2 - s * x2;   // q2 *= e^{-i phi}
    }
}

// Amplitudes of a qutrit record (the first 48 of its 64 bytes).
// Elitism (Sec. IV-E.1) of a used slot whose segment fitness is v: strictly
// better -> the state becomes the best, otherwise the best state is restored.
// Returns whether the best copy changed.
__device__ __forceinline__ bool elitism(float v, SlotRec& r, QState& q, bool rot) {
    if (v > r.best_f) {
        r.best_f = v;
        r.best_theta = r.theta;
        if (rot)
#pragma unroll
            for (int c = 0; c < 6; ++c) q.bq[c] = q.q[c];
        return true;
    }
    r.theta = r.best_theta;
    if (rot)
#pragma unroll
        for (int c = 0; c < 6; ++c) q.q[c] = q.bq[c];
    return false;
}

// The elitism of a slot that no other circuit of the generation used, with
// its circuit's fitness v as the segment fitness: run by that circuit as soon
// as its fitness is known, from the records it gathered (nothing else writes
// them before the update).  Only what changes is written; the key stays 0,
// so the update sees the slot as unused.
__device__ __forceinline__ void commit_alone(const LoopArgs& a, uint32_t i, uint32_t s, float v, SlotFull f) {
    const size_t o = (size_t)i * a.S + s, oq = (size_t)i * a.Q + s;
    const bool rot = s < a.Q;
    SlotRec r = f.r;
    QState q = f.q;                         // (a template slot's is never stored)
    const uint32_t th = r.theta;
    bool qsame = true;
#pragma unroll
    for (int c = 0; c < 6; ++c) qsame = qsame && __float_as_uint(q.q[c]) == __float_as_uint(q.bq[c]);
    const bool better = elitism(v, r, q, rot);
    if (better || r.theta != th) a.slot[o] = r;
    if (rot && !qsame) store_qstate(a.qrec + oq, q);
}

// Mutation of one slot (Sec. IV-F) with its own draw; segFit is the slot's
// best fitness (0 if never used).  Qubit mode: theta +- floor((1 - segFit) *
// range); qutrit mode: one SU(3) parameter step.
__device__ __forceinline__ void mutate_state(const LoopArgs& a, uint32_t gen, uint32_t i, uint32_t s,
                                             bool qutrit_mode, SlotRec& r, QState& q) {
    const float seg = r.best_f < 0.0f ? 0.0f : r.best_f;
    const float om = 1.0f - seg;
    const u32x4 w = draw(a.seed, TAG_MUT_SLOT, gen, i, s);
    if (!qutrit_mode) {
        const uint32_t d = (uint32_t)floorf(om * a.r32);
        r.theta = (w.x & 1u) ? r.theta - d : r.theta + d;
    } else {
        const int j = (int)scale_u32(w.y, 8u);
        const float u = (float)(w.z >> 8) * 0x1p-24f;
        const float x = u * om;
        const int ai = (int)floorf(x * 4096.0f);
        su3_step(q.q, j, ai, a.su3_tab);
    }
}

// The slots of a generation and which of them more than one circuit uses:
// one workgroup per population draws every (circuit, position) entry's slot
// (the generation's SAMPLE stream) and enters it in an LDS hash table (open
// addressing, at most half full; bit 31 of an entry marks a slot entered
// twice), then writes each entry's slot word (the slot index, bit 31 set if
// the slot is shared) and the list of the shared entries.  The fused kernel
// takes its slots from the words and commits the elitism of the unshared
// ones itself (commit_alone); the shared ones keep the largest key for the
// update, whose part A walks the list.  Used
// when a population has at most DEDUP_MAX_ENTRIES entries of at most 256
// positions and fewer than 2^31 slots.  The slots drawn depend on the seed and
// the generation alone, not on the encoding, so the search of a generation
// can run before the previous generation has been updated: the update kernel
// runs it for the next generation (its part D), and dedup_kernel serves a
// generation with no update before it.
__device__ __forceinline__ uint32_t dedup_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x45D9F3Bu;
    x ^= x >> 16;
    return x;
}

// Population i's search, by a whole workgroup of 256 threads, with keys the
// dedup_table(P * L) words of dynamic LDS.
__device__ __forceinline__ void dedup_population(const LoopArgs& a, uint32_t gen, uint32_t i,
                                                 uint32_t* keys) {
    constexpr uint32_t EMPTY = 0xFFFFFFFFu;
    constexpr int PER = DEDUP_MAX_ENTRIES / 256;
    const uint32_t L = (uint32_t)a.L, LP = L * (uint32_t)a.P, T = dedup_table(LP);
    for (uint32_t t = threadIdx.x; t < T; t += 256) keys[t] = EMPTY;
    __syncthreads();
    uint32_t sl[PER], at[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t e = (uint32_t)u * 256u + threadIdx.x;
        sl[u] = 0u;
        at[u] = 0u;
        if (e >= LP) continue;
        const uint32_t s = sample_slot(a, gen, i, e / L, e % L);      // < 2^31
        uint32_t h = (uint32_t)(((uint64_t)dedup_hash(s) * T) >> 32);
        // the table holds at most LP <= T / 2 slots: a free entry is always
        // found
        while (true) {
            const uint32_t prev = atomicCAS(&keys[h], EMPTY, s);
            if (prev == EMPTY) break;
            if ((prev & ~DUP_SHARED) == s) {
                atomicOr(&keys[h], DUP_SHARED);
                break;
            }
            h = h + 1u == T ? 0u : h + 1u;
        }
        sl[u] = s;
        at[u] = h;
    }
    __shared__ uint32_t n_shared;
    if (threadIdx.x == 0) n_shared = 0u;
    __syncthreads();
    const size_t base = (size_t)(gen & 1u) * a.I + i;
    uint32_t* out = dup_words(a, gen) + (size_t)i * LP;
    uint2* list = a.shared_list + base * LP;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t e = (uint32_t)u * 256u + threadIdx.x;
        if (e >= LP) continue;
        const uint32_t sh = keys[at[u]] & DUP_SHARED;
        out[e] = sl[u] | sh;
        // the shared entries, for the update (in no particular order: each
        // entry's work on its slot does not depend on the others')
        if (sh) list[atomicAdd(&n_shared, 1u)] = make_uint2(e, sl[u]);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.shared_count[base] = n_shared;
}

__global__ __launch_bounds__(256) void dedup_kernel(LoopArgs a, uint64_t gen64) {
    extern __shared__ __align__(16) uint32_t dedup_keys[];
    dedup_population(a, gen_of(a, gen64), blockIdx.x, dedup_keys);
}

// Part C: the instance's best circuit of the generation (largest f, lowest
// index; NaN never counts) updates its best circuit ever.  Part A: the used
// slots the mutation leaves alone (those of individuals that do not mutate,
// and the template slots of individuals mutating in qutrit mode), one thread
// per (circuit, position) entry, or, after the shared-slot search, per entry
// of the population's list of shared entries (the fused kernel committed
// the rest); an entry handles its slot only if its circuit holds the slot's
// key.  Part B: the slots the mutation moves (qubit
// mode: every slot of the individual; qutrit mode: its rotation slots), one
// thread per slot, since the individual's slots belong to nobody else:
// elitism if the slot was used, then mutation.  Part D (optional): the
// shared-slot search of the next generation, one workgroup per population
// (a launch fewer per generation than a kernel of its own).  The
// grid holds part C, then part B (the longest chains), then part D, then
// part A, so the longer work is dispatched first.
constexpr int UPD_BLOCK = 256;
constexpr int UPD_MAX_P = 16384;          // part B's list of mutated individuals lives in LDS
constexpr int UPD_WPB = UPD_BLOCK / 64;   // wavefronts per workgroup
// part B: SPL slots per lane of an item (64 SPL slots, one wavefront): 4
// when many populations fill the launch (2 and 8 measured slower), 1 for a
// few large populations, which need the wavefronts

// Entry idx (= i * P * L + k * L + pos) of population i, whose slot is s.
__device__ __forceinline__ void part_a_entry(const LoopArgs& a, uint32_t gen, uint32_t i, uint32_t idx,
                                             uint32_t s, const float* __restrict__ f) {
    const uint32_t L = (uint32_t)a.L, LP = L * (uint32_t)a.P;
    const float fk = f[idx / L];                // the entry's circuit's fitness
    if (s >= a.S) return;
    const uint32_t ind = (s % LP) / L;
    const size_t o = (size_t)i * a.S + s, oq = (size_t)i * a.Q + s;
    const bool rot = s < a.Q;
    SlotRec r = a.slot[o];
    QState q{};
    if (rot) q = load_qstate(a.qrec + oq);      // issued before ownership is known
    // the individual's mutation decision, from the generation's decision mask
    // (its word is loaded with the records)
    const uint32_t mw = mask_of(a, gen, i)[ind >> 5];
    const bool mut = ((mw >> (ind & 31u)) & 1u) != 0u;
    // the entry takes the slot if its circuit's fitness is the slot's segment
    // fitness (when several circuits share that fitness, each applies the
    // same elitism to the same record, which leaves the same state)
    if (r.key == 0u || !(fk >= 0.0f) || r.key != seg_key(fk)) return;
    if (mut) {
        // part B takes the slots the mutation moves: every slot of an
        // individual in qubit mode, the rotation slots in qutrit mode
        bool qm;
        mutates(a, gen, i, ind, &qm);
        if (!qm || rot) return;
    }
    const float v = seg_fitness(r.key);
    r.key = 0u;
    elitism(v, r, q, rot);
    a.slot[o] = r;
    if (rot) store_qstate(a.qrec + oq, q);
}

// One thread per entry (idx over all populations' entries): slots NULL
// draws the entry's slot again (the generation's own sampling, which saves
// a dependent load); otherwise it is read.
__device__ __forceinline__ void update_part_a(const LoopArgs& a, uint32_t gen, uint32_t idx,
                                              const uint32_t* __restrict__ slots,
                                              const float* __restrict__ f) {
    const uint32_t L = (uint32_t)a.L, LP = L * (uint32_t)a.P;
    if (idx >= (uint32_t)a.I * LP) return;
    const uint32_t i = idx / LP, k = (idx % LP) / L;
    part_a_entry(a, gen, i, idx, slots ? slots[idx] : sample_slot(a, gen, i, k, idx % L), f);
}

// With the shared-slot search (the fused kernel committed the slots one
// circuit alone used): one workgroup per population over its list of shared
// entries.
__device__ __forceinline__ void update_part_a_shared(const LoopArgs& a, uint32_t gen, uint32_t i,
                                                     const float* __restrict__ f) {
    const size_t base = (size_t)(gen & 1u) * a.I + i;
    const uint32_t n = a.shared_count[base], LP = (uint32_t)a.L * (uint32_t)a.P;
    const uint2* list = a.shared_list + base * LP;
    for (uint32_t t = threadIdx.x; t < n; t += UPD_BLOCK) {
        const uint2 es = list[t];
        part_a_entry(a, gen, i, i * LP + es.x, es.y, f);
    }
}

// Workgroup b of part B serves instance b / per_inst: it lists the
// instance's mutated individuals in LDS from the decision mask, then its
// wavefronts walk the (individual, chunk of 64 SPL slots) items, one item
// each, with stride per_inst * UPD_WPB.
template <int SPL>
__device__ __forceinline__ void update_part_b(const LoopArgs& a, uint32_t gen, uint32_t b,
                                              uint32_t per_inst) {
    extern __shared__ uint16_t list[];        // P entries (launch-time size)
    __shared__ uint32_t total;
    const uint32_t L = (uint32_t)a.L, P = (uint32_t)a.P, LP = L * P;
    const uint32_t per = a.R * L;                               // slots of one individual
    constexpr uint32_t ITEM = 64u * SPL;
    const uint32_t chunks = (per + ITEM - 1) / ITEM;
    const uint32_t i = b / per_inst;
    if (i >= (uint32_t)a.I) return;
    if (threadIdx.x < 64) {
        // wave 0: prefix count over the mask words, 64 at a time (all the
        // words, at most UPD_MAX_P / 32, are loaded first)
        constexpr int MAXW = UPD_MAX_P / 32 / 64;
        const uint32_t* mask = mask_of(a, gen, i);
        const int lane = (int)threadIdx.x;
        uint32_t words[MAXW];
#pragma unroll
        for (int q = 0; q < MAXW; ++q) {
            const uint32_t w = (uint32_t)(q * 64 + lane);
            words[q] = w < a.MW ? mask[w] : 0u;
        }
        uint32_t base = 0;
#pragma unroll
        for (int q = 0; q < MAXW; ++q) {
            if ((uint32_t)(q * 64) >= a.MW) break;
            const uint32_t w = (uint32_t)(q * 64 + lane);
            uint32_t bits = words[q];
            if (w == a.MW - 1 && (P & 31u)) bits &= (1u << (P & 31u)) - 1u;
            const uint32_t c = (uint32_t)__popc(bits);
            uint32_t incl = c;                  // inclusive scan over the wave
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = (uint32_t)__shfl_up((int)incl, d, 64);
                if (lane >= d) incl += o;
            }
            uint32_t pos = base + incl - c;
            while (bits) {
                const int bit = __ffs(bits) - 1;
                list[pos++] = (uint16_t)(w * 32u + (uint32_t)bit);
                bits &= bits - 1u;
            }
            base += (uint32_t)__shfl((int)incl, 63, 64);
        }
        if (lane == 0) total = base;
    }
    __syncthreads();
    const uint32_t count = total;
    // one (individual, chunk) item per wavefront, SPL slots per lane with
    // their loads issued together
    const uint32_t wv = threadIdx.x >> 6, ln = threadIdx.x & 63u;
    for (uint32_t t = (b % per_inst) * UPD_WPB + wv; t < count * chunks; t += per_inst * UPD_WPB) {
        // (the wavefront serves one individual: its decision is drawn once,
        // on the scalar unit)
        const uint32_t ind = (uint32_t)__builtin_amdgcn_readfirstlane((int)list[t / chunks]);
        bool qm;
        mutates(a, gen, i, ind, &qm);
        SlotRec r[SPL];
        QState q[SPL];
        uint32_t sl[SPL];
        bool act[SPL];
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            const uint32_t e = (t % chunks) * ITEM + (uint32_t)u * 64u + ln;
            const uint32_t r_ = e / L, pos = e - r_ * L;
            sl[u] = r_ * LP + ind * L + pos;
            const bool rot = r_ < (uint32_t)a.n;
            // qutrit mode moves only the rotation slots; the others'
            // elitism is part A's
            act[u] = e < per && !(qm && !rot);
            q[u] = QState{};
            if (act[u]) {
                r[u] = a.slot[(size_t)i * a.S + sl[u]];
                if (rot && qm) q[u] = load_qstate(a.qrec + (size_t)i * a.Q + sl[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            if (!act[u]) continue;
            const uint32_t s = sl[u];
            const size_t o = (size_t)i * a.S + s, oq = (size_t)i * a.Q + s;
            const bool rot = s < a.Q;
            const bool used = r[u].key != 0u;
            // qubit mode reads a rotation slot's qutrit only for its elitism
            if (rot && !qm && used) q[u] = load_qstate(a.qrec + oq);
            if (used) elitism(seg_fitness(r[u].key), r[u], q[u], rot);
            r[u].key = 0u;
            mutate_state(a, gen, i, s, qm, r[u], q[u]);
            // an unused slot in qutrit mode keeps its record (only the qutrit moves)
            if (used || !qm) a.slot[o] = r[u];
            if (rot && (used || qm)) store_qstate(a.qrec + oq, q[u]);
        }
    }
}

// Wavefronts per instance in part C: each lane scans at most 16 fitness
// values per pass (P <= 1024: 1, P <= 2048: 2, else 4).
__host__ __device__ inline int part_c_waves(int P) { return P > 2048 ? 4 : (P > 1024 ? 2 : 1); }

__device__ __forceinline__ void update_part_c(const LoopArgs& a, uint32_t b,
                                              const uint16_t* __restrict__ gates,
                                              const uint32_t* __restrict__ angles,
                                              const float* __restrict__ f) {
    __shared__ float cbest[4];
    __shared__ uint32_t cidx[4];
    const uint32_t L = (uint32_t)a.L, P = (uint32_t)a.P;
    const int cw = part_c_waves(a.P);
    const int lane = (int)lane_id(), wave = (int)(threadIdx.x >> 6), sub = wave % cw;
    const uint32_t i = b * (uint32_t)(4 / cw) + (uint32_t)(wave / cw);
    float best = -1.0f;
    uint32_t bk = 0xFFFFFFFFu;
    if (i < (uint32_t)a.I) {
        const float* fi = f + (size_t)i * P;
        const uint32_t step = 64u * (uint32_t)cw;
        for (uint32_t k0 = (uint32_t)(sub * 64 + lane); k0 < P; k0 += 16 * step) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t k = k0 + (uint32_t)j * step;
                v[j] = k < P ? fi[k] : -1.0f;
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (v[j] > best) { best = v[j]; bk = k0 + (uint32_t)j * step; }
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const float ob = __shfl_xor(best, m, 64);
        const uint32_t ok = (uint32_t)__shfl_xor((int)bk, m, 64);
        if (ob > best || (ob == best && ok < bk)) { best = ob; bk = ok; }
    }
    if (cw > 1) {
        if (lane == 0) { cbest[wave] = best; cidx[wave] = bk; }
        __syncthreads();
        if (sub != 0) return;
        for (int w = 1; w < cw; ++w) {
            const float ob = cbest[wave + w];
            const uint32_t ok = cidx[wave + w];
            if (ob > best || (ob == best && ok < bk)) { best = ob; bk = ok; }
        }
    }
    if (i >= (uint32_t)a.I || bk == 0xFFFFFFFFu || !(best > a.inst_best_f[i])) return;
    const size_t row = ((size_t)i * P + bk) * L;
    for (uint32_t l = lane; l < L; l += 64) {
        a.inst_best_gates[(size_t)i * L + l] = gates[row + l];
        if (angles) a.inst_best_angles[(size_t)i * L + l] = angles[row + l];
    }
    if (lane == 0) a.inst_best_f[i] = best;
}

template <int SPL>
__global__ __launch_bounds__(UPD_BLOCK) void qeqea_update_kernel(LoopArgs a, uint64_t gen64,
                                                                 const uint32_t* __restrict__ slots,
                                                                 const uint16_t* __restrict__ gates,
                                                                 const uint32_t* __restrict__ angles,
                                                                 const float* __restrict__ f,
                                                                 uint32_t nC, uint32_t nB, uint32_t nD,
                                                                 uint32_t per_inst, bool shared) {
    const uint32_t gen = gen_of(a, gen64);
    // parts D and A start at multiples of 8, so that a block's XCD is its
    // index within the part modulo 8
    const uint32_t d0 = (nC + nB + 7u) & ~7u;
    const uint32_t a0 = (d0 + nD + 7u) & ~7u;
    if (blockIdx.x < nC) {
        update_part_c(a, blockIdx.x, gates, angles, f);
    } else if (blockIdx.x < nC + nB) {
        update_part_b<SPL>(a, gen, blockIdx.x - nC, per_inst);
    } else if (blockIdx.x >= d0 && blockIdx.x < d0 + nD) {
        // part D: the shared-slot search of the next generation (its words go
        // to the other buffer), each population's on the XCD whose L2 the
        // fused kernel will read them from
        extern __shared__ __align__(16) uint32_t dedup_keys[];
        dedup_population(a, gen + 1u, xcd_swizzle(blockIdx.x - d0, nD), dedup_keys);
    } else if (blockIdx.x >= a0) {
        // part A: each XCD takes the circuits the fused kernel ran on it,
        // from the last back (the records touched last are the likeliest to
        // still be cached)
        const uint32_t nA = gridDim.x - a0;
        if (shared) {
            update_part_a_shared(a, gen, xcd_swizzle(blockIdx.x - a0, nA), f);
        } else {
            const uint32_t blk = nA - 1u - xcd_swizzle(blockIdx.x - a0, nA);
            update_part_a(a, gen, blk * UPD_BLOCK + threadIdx.x, slots, f);
        }
    }
}

// Dense copy of one field of the encoding state.
__global__ void state_gather_kernel(LoopArgs a, int which, void* __restrict__ dst) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (which == 0 || which == 2 || which == 3) {
        if (idx >= (size_t)a.I * a.S) return;
        const SlotRec r = a.slot[idx];
        if (which == 0) static_cast<uint32_t*>(dst)[idx] = r.theta;
        else if (which == 2) static_cast<float*>(dst)[idx] = r.best_f;
        else static_cast<uint32_t*>(dst)[idx] = r.best_theta;
    } else {
        if (idx >= (size_t)a.I * a.Q * 6) return;
        const QutritRec& q = a.qrec[idx / 6];
        static_cast<float*>(dst)[idx] = which == 1 ? q.q[idx % 6] : q.bq[idx % 6];
    }
}

// ----------------------------------------------------------------------- GA
// One workgroup per population: SUS over integer weights floor(f * 2^24),
// two-point crossover of children j and j + P/2, gene mutation, and the best
// parent copied unchanged into child 0.  Reads genomes[gen & 1], writes
// genomes[(gen + 1) & 1].
constexpr int GA_MAX_P = 4096;

__global__ __launch_bounds__(256) void ga_update_kernel(LoopArgs a, uint64_t gen64,
                                                        const float* __restrict__ f) {
    __shared__ unsigned long long pre[GA_MAX_P + 1];
    __shared__ int32_t sel[GA_MAX_P];
    __shared__ float bestv[4];
    __shared__ int besti[4];
    const uint32_t gen = gen_of(a, gen64);
    const uint32_t i = blockIdx.x;
    const int P = a.P, tid = threadIdx.x, nt = blockDim.x;
    // population i's width, genome length and genomes (mixed populations
    // carry their own)
    const int n = a.inst_n ? a.inst_n[i] : a.n, L = a.inst_L ? a.inst_L[i] : a.L;
    const size_t base = a.inst_goff ? (size_t)a.inst_goff[i] : (size_t)i * P * L;
    const uint16_t* cur = a.genomes[gen & 1] + base;
    uint16_t* nxt = a.genomes[(gen + 1) & 1] + base;
    const float* fi = f + (size_t)i * P;
    // weights and best (lowest index among the maxima)
    float best = -1.0f;
    int bi = 0x7FFFFFFF;
    for (int k = tid; k < P; k += nt) {
        const float v = fi[k];
        pre[k + 1] = (v >= 0.0f) ? (unsigned long long)(uint32_t)floorf(v * 16777216.0f) : 0ull;
        if (v > best) { best = v; bi = k; }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        const float ob = __shfl_xor(best, m, 64);
        const int oi = __shfl_xor(bi, m, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if ((tid & 63) == 0) { bestv[tid >> 6] = best; besti[tid >> 6] = bi; }
    if (tid == 0) pre[0] = 0;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < (nt >> 6); ++w)
            if (bestv[w] > best || (bestv[w] == best && besti[w] < bi)) { best = bestv[w]; bi = besti[w]; }
        bestv[0] = best; besti[0] = bi;
        // inclusive prefix (serial: P <= 4096 additions)
        for (int k = 1; k <= P; ++k) pre[k] += pre[k - 1];
        if (pre[P] == 0)
            for (int k = 0; k <= P; ++k) pre[k] = (unsigned long long)k;
    }
    __syncthreads();
    best = bestv[0];
    bi = besti[0] == 0x7FFFFFFF ? 0 : besti[0];
    const unsigned long long W = pre[P];
    const uint32_t w0 = draw(a.seed, TAG_GA_SUS, gen, i, 0u).x;
    const unsigned long long r = (unsigned long long)w0 * (W >> 32) +
                                 (((unsigned long long)w0 * (W & 0xFFFFFFFFull)) >> 32);
    for (int k = tid; k < P; k += nt) {
        const unsigned long long ptr = (r + (unsigned long long)k * W) / (unsigned long long)P;
        int lo = 0, hi = P - 1;        // first m with pre[m + 1] > ptr
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid + 1] > ptr) hi = mid; else lo = mid + 1;
        }
        sel[k] = lo;
    }
    __syncthreads();
    for (size_t e = tid; e < (size_t)P * L; e += nt) {
        const int k = (int)(e / L), pos = (int)(e % L);
        nxt[e] = cur[(size_t)sel[k] * L + pos];
    }
    __syncthreads();
    const int half = P / 2;
    for (int j = tid; j < half; j += nt) {
        const u32x4 w = draw(a.seed, TAG_GA_XOVER, gen, i, (uint32_t)j);
        if (!((uint64_t)w.x < a.thr_pc)) continue;
        const int c1 = (int)scale_u32(w.y, (uint32_t)(L + 1)), c2 = (int)scale_u32(w.z, (uint32_t)(L + 1));
        const int lo = min(c1, c2), hi = max(c1, c2);
        for (int pos = lo; pos < hi; ++pos) {
            const uint16_t t = nxt[(size_t)j * L + pos];
            nxt[(size_t)j * L + pos] = nxt[(size_t)(j + half) * L + pos];
            nxt[(size_t)(j + half) * L + pos] = t;
        }
    }
    __syncthreads();
    const uint32_t nl = (uint32_t)lib_size(a.lib, n);
    for (size_t e = tid; e < (size_t)P * L; e += nt) {
        const u32x4 w = draw(a.seed, TAG_GA_MUT, gen, i, (uint32_t)e);
        if ((uint64_t)w.x < a.thr_pg) nxt[e] = lib_desc(a.lib, n, (int)scale_u32(w.y, nl));
    }
    __syncthreads();
    for (int pos = tid; pos < L; pos += nt) nxt[pos] = cur[(size_t)bi * L + pos];
    // best circuit ever seen by this population (rows of a.L entries)
    if (best > a.inst_best_f[i]) {
        for (int pos = tid; pos < L; pos += nt)
            a.inst_best_gates[(size_t)i * a.L + pos] = cur[(size_t)bi * L + pos];
        __syncthreads();
        if (tid == 0) a.inst_best_f[i] = best;
    }
}

// --------------------------------------------------------------- elite FP64
// Top-k circuits of each population by (f descending, index ascending), as
// ascending 64-bit keys (NaN and padding last).  Bitonic sorts of four keys
// per thread: exchanges at strides 1 and 2 stay in a thread's registers,
// strides 4..128 within a wavefront (shuffles of the partner lane), and only
// strides of 256 and more go through LDS with workgroup barriers.
//   tiles: one wavefront per 256 circuits sorts its tile; with one tile it
//          writes the result, otherwise its first k keys (k <= 64);
//   merge: one workgroup per population sorts the tiles' candidates;
//   whole: one workgroup per population sorts all P keys (k > 64).
// Spreading the tiles over the GPU keeps the common case (k = 32 of 4096)
// off a single compute unit.
constexpr int ELITE_TILE = 256;
constexpr int ELITE_MAX_TILE_K = 64;
enum EliteMode { ELITE_TILES = 0, ELITE_MERGE = 1, ELITE_WHOLE = 2 };

__device__ __forceinline__ unsigned long long cas_keep(unsigned long long v, unsigned long long p,
                                                       bool lower, bool asc) {
    // the element at the lower index of an ascending pair keeps the minimum
    const bool take_min = lower == asc;
    return take_min ? (p < v ? p : v) : (p > v ? p : v);
}

__device__ __forceinline__ unsigned long long elite_key(float x, uint32_t c) {
    // non-negative floats order like their bit patterns; NaN last
    const uint32_t ord = (x >= 0.0f) ? __float_as_uint(x) + 1u : 0u;
    return ((unsigned long long)(0xFFFFFFFFu - ord) << 32) | c;
}

// Ascending bitonic sort of the 4 * blockDim.x keys held four per thread
// (key 4 * tid + q in v[q]); blockDim.x is a power of two >= 64 and lds holds
// 4 * blockDim.x keys.
__device__ __forceinline__ void bitonic_sort4(unsigned long long v[4], unsigned long long* lds) {
    const int tid = threadIdx.x, nk = 4 * (int)blockDim.x;
    for (int size = 2; size <= nk; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= 256) {
#pragma unroll
                for (int q = 0; q < 4; ++q) lds[4 * tid + q] = v[q];
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * tid + q;
                    v[q] = cas_keep(v[q], lds[e ^ stride], (e & stride) == 0, (e & size) == 0);
                }
                __syncthreads();
            } else if (stride >= 4) {
                const int lm = stride >> 2;          // partner lane offset
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * tid + q;
                    const unsigned long long p = __shfl_xor(v[q], lm, 64);
                    v[q] = cas_keep(v[q], p, (e & stride) == 0, (e & size) == 0);
                }
            } else {
                unsigned long long w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * tid + q;
                    w[q] = cas_keep(v[q], v[q ^ stride], (e & stride) == 0, (e & size) == 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = w[q];
            }
        }
    }
}

// T: tiles per population; cand: [I][T][k] keys (tiles and merge, T > 1).
template <int MODE>
__global__ __launch_bounds__(1024) void elite_select_kernel(LoopArgs a, const float* __restrict__ f,
                                                           int k, int T, unsigned long long* cand,
                                                           int32_t* __restrict__ idx_out) {
    extern __shared__ unsigned long long elite_lds[];
    const int tid = threadIdx.x, P = a.P;
    const int i = MODE == ELITE_TILES ? (int)blockIdx.x / T : (int)blockIdx.x;
    const int t = MODE == ELITE_TILES ? (int)blockIdx.x % T : 0;
    unsigned long long v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = 4 * tid + q;
        unsigned long long kv = ~0ull;
        if constexpr (MODE == ELITE_MERGE) {
            if (e < T * k) kv = cand[(size_t)i * T * k + e];
        } else {
            const int c = t * ELITE_TILE + e;     // (whole: t = 0, e over the population)
            if (c < P) kv = elite_key(f[(size_t)i * P + c], (uint32_t)c);
        }
        v[q] = kv;
    }
    bitonic_sort4(v, elite_lds);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = 4 * tid + q;
        if (e >= k) continue;
        if (MODE == ELITE_TILES && T > 1) cand[((size_t)i * T + t) * k + e] = v[q];
        else idx_out[(size_t)i * k + e] = (int32_t)(v[q] & 0xFFFFFFFFu);
    }
}

__global__ __launch_bounds__(256) void elite_eval_kernel(LoopArgs a, const uint16_t* __restrict__ gates,
                                                         const uint32_t* __restrict__ angles,
                                                         int k, const int32_t* __restrict__ idx,
                                                         double* __restrict__ f64) {
    const int i = blockIdx.x / k, e = blockIdx.x % k;
    const int c = idx[(size_t)i * k + e];
    uint32_t err = (c < 0 || c >= a.P) ? (uint32_t)QE_DEVERR_RANGE : 0u;
    const int n = a.inst_n ? a.inst_n[i] : a.n, L = a.inst_L ? a.inst_L[i] : a.L;
    const size_t row = (a.inst_goff ? (size_t)a.inst_goff[i] : (size_t)i * a.P * L) + (size_t)(err ? 0 : c) * L;
    const double* T = a.target64 + 2 * (a.inst_toff ? (size_t)a.inst_toff[i] : (size_t)i << (2 * n));
    double* Mr = generic_lds<double>();         // dynamic LDS for the context's largest width
    lds_generic_body<double, false>(n, L, gates + row, angles ? angles + row : nullptr, T, err,
                                    f64 + blockIdx.x, nullptr, nullptr, nullptr, a.err, a.fit_mode,
                                    Mr, Mr + ((size_t)1 << (2 * a.n)));
}

// FP64 re-check of elite circuits of width NQ (4 or 5) over a discrete
// library: W wavefronts per circuit (each owning N / W columns: gates mix
// rows only, so the wavefronts of a circuit never exchange data until the
// reduction), CPB circuits per workgroup, the product U T^dagger (Eq. 11)
// as complex128 in LDS.  Lane l of a wavefront owns column
// j = w N / W + l mod (N / W) and row group h = l div (N / W); a gate's row
// pairs are its pair indices (the target bit taken out) or, for a
// controlled gate, its quad indices (target and control bits taken out),
// the row group supplying the low bits.  NOT and CNOT move no data: as in
// the FP32 LDS path, logical row r is stored at row A r ^ b (A's column p in
// bits 6p..6p+5), and they only update A and b.  CV and CV+ take the halves
// of a + b and i (a - b); H and T are applied as their matrices say.  The
// results agree with the generic FP64 body to rounding.
template <int NQ, int W>
struct Elite64Layout {
    static constexpr int N = 1 << NQ, LPR = N / W, RG = 64 / LPR;
    static constexpr int RGB = RG == 2 ? 1 : (RG == 4 ? 2 : 3);
    static_assert(RG == (1 << RGB) && RG <= 8, "row groups");
    static_assert(NQ - 2 >= RGB, "a controlled gate's quads cover the row groups");
};

// One gate on the lane's pairs: base = stored row of the lane's first pair
// (row group bits, control row and the map's translation folded in), pass[k]
// = stored image of pair-index bit RGB + k, tstep = stored image of the
// target bit.
template <int NQ, int W, bool CTL>
__device__ __forceinline__ void elite64_pairs(double2* M, int kind, uint32_t base, const uint32_t* pass,
                                              uint32_t tstep, int j) {
    using LY = Elite64Layout<NQ, W>;
    constexpr int QB = NQ - 1 - (CTL ? 1 : 0);       // bits of the pair index
    constexpr int NP = (1 << QB) / LY::RG;           // pairs per lane
    double2 X[NP], Y[NP];
    int o0[NP], o1[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        uint32_t sr = base;
#pragma unroll
        for (int k = 0; (1 << k) < NP; ++k)
            if ((m >> k) & 1) sr ^= pass[k];
        o0[m] = (int)((sr << NQ) | (uint32_t)j);
        o1[m] = (int)(((sr ^ tstep) << NQ) | (uint32_t)j);
        X[m] = M[o0[m]];
        Y[m] = M[o1[m]];
    }
    constexpr double S2 = 0.70710678118654752440084436210485;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const double2 a = X[m], bb = Y[m];
        double2 x, y;
        if (CTL) {
            // V = [[1+i, 1-i], [1-i, 1+i]] / 2: a' = (s + i d) / 2, b' = (s - i d) / 2
            // with s = a + b, d = a - b; V+ swaps the two
            const double sr = 0.5 * (a.x + bb.x), si = 0.5 * (a.y + bb.y);
            const double dr = 0.5 * (a.x - bb.x), di = 0.5 * (a.y - bb.y);
            const double2 p = make_double2(sr - di, si + dr), q = make_double2(sr + di, si - dr);
            x = kind == KIND_CV ? p : q;
            y = kind == KIND_CV ? q : p;
        } else if (kind == KIND_H) {
            x = make_double2(S2 * (a.x + bb.x), S2 * (a.y + bb.y));
            y = make_double2(S2 * (a.x - bb.x), S2 * (a.y - bb.y));
        } else {   // T: b' = b (1 + i) / sqrt 2
            x = a;
            y = make_double2(S2 * (bb.x - bb.y), S2 * (bb.x + bb.y));
        }
        M[o0[m]] = x;
        M[o1[m]] = y;
    }
}

template <int NQ, int W, int CPB>
__global__ __launch_bounds__(64 * W * CPB) void elite64_kernel(LoopArgs a, const uint16_t* __restrict__ gates,
                                                               int k, const int32_t* __restrict__ idx,
                                                               double* __restrict__ f64) {
    using LY = Elite64Layout<NQ, W>;
    constexpr int N = LY::N, LPR = LY::LPR, RG = LY::RG, RGB = LY::RGB;
    __shared__ double2 Ms[CPB][N * N];
    __shared__ double red[CPB][W];
    const int wave = (int)(threadIdx.x >> 6), lane = (int)lane_id();
    const int circ = wave / W, wv = wave % W;
    const uint32_t ci = __builtin_amdgcn_readfirstlane(blockIdx.x * CPB + (uint32_t)circ);
    const bool valid = ci < (uint32_t)a.I * (uint32_t)k;   // (every wavefront reaches the barrier)
    const uint32_t i = valid ? ci / (uint32_t)k : 0u;
    const int c = valid ? idx[ci] : 0;
    uint32_t err = (c < 0 || c >= a.P) ? (uint32_t)QE_DEVERR_RANGE : 0u;
    const int L = a.L;
    const uint16_t* g = gates + ((size_t)i * a.P + (size_t)(err ? 0 : c)) * L;
    const double2* T = reinterpret_cast<const double2*>(a.target64) + ((size_t)i << (2 * NQ));
    double2* M = Ms[circ];
    const int j = wv * LPR + lane % LPR, h = lane / LPR;
    uint64_t A = 0;                                   // the row map, identity
#pragma unroll
    for (int p = 0; p < NQ; ++p) A |= (uint64_t)(1u << p) << (6 * p);
    uint32_t b = 0;
    bool ok = valid && err == 0;
    if (ok) {
        // M = T^dagger on this wavefront's columns: M[r][j] = conj(T[j][r])
#pragma unroll
        for (int m = 0; m < N / RG; ++m) {
            const int r = h + m * RG;
            const double2 t = T[(size_t)j * N + r];
            M[r * N + j] = make_double2(t.x, -t.y);
        }
        wave_lds_fence();
        for (int l0 = 0; l0 < L && ok; l0 += 64) {
            // the chunk's gate program, one gate per lane: descriptor checks,
            // the row map in force at each gate (NOT and CNOT folded in, in
            // circuit order), and each data-moving gate's stored offsets
            const int cnt = min(64, L - l0);
            const bool in = lane < cnt;
            const uint32_t dv = in ? (uint32_t)g[l0 + lane] : 0u;
            if (__ballot(in && !desc_valid(dv, NQ))) { ok = false; break; }
            const int kind = (int)(dv & 15u);
            const int tp = NQ - 1 - (int)((dv >> 4) & 15u), cp = NQ - 1 - (int)((dv >> 8) & 15u);
            const bool perm = in && (kind == KIND_NOT || kind == KIND_CNOT);
            uint64_t myA = A;
            uint32_t myB = b;
            uint64_t pm = __ballot(perm);
            while (pm) {
                const int gg = (int)__builtin_ctzll(pm);
                pm &= pm - 1;
                const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)dv, gg);
                const int pt = NQ - 1 - (int)((d >> 4) & 15u);
                const uint32_t colt = (uint32_t)(A >> (6 * pt)) & 63u;
                if ((d & 15u) == (uint32_t)KIND_NOT) {
                    b ^= colt;
                } else {
                    const int pc = NQ - 1 - (int)((d >> 8) & 15u);
                    A ^= (uint64_t)colt << (6 * pc);
                }
                if (lane > gg) { myA = A; myB = b; }
            }
            const bool live = in && kind != KIND_I && !perm;
            const bool ctl = kind == KIND_CV || kind == KIND_CVDG;
            auto col = [&](int p) -> uint32_t { return (uint32_t)(myA >> (6 * (p & 7))) & 63u; };
            const int lo = ctl ? min(tp, cp) : tp, hi = ctl ? max(tp, cp) : NQ;
            auto img = [&](int kk) -> uint32_t {       // pair-index bit kk -> stored row bits
                int pos = kk < lo ? kk : kk + 1;
                pos = pos < hi ? pos : pos + 1;
                return col(pos);
            };
            const uint32_t gbase = live ? (myB ^ (ctl ? col(cp) : 0u)) : 0u;
            const uint32_t gt = live ? col(tp) : 0u;
            uint32_t gimg[NQ - 1];
#pragma unroll
            for (int kk = 0; kk < NQ - 1; ++kk) gimg[kk] = live ? img(kk) : 0u;
            uint64_t todo = __ballot(live);
            while (todo) {
                const int gg = (int)__builtin_ctzll(todo);
                todo &= todo - 1;
                auto rl = [&](uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, gg); };
                const int kg = (int)rl((uint32_t)kind);
                uint32_t base = rl(gbase);
                uint32_t im[NQ - 1];
#pragma unroll
                for (int kk = 0; kk < NQ - 1; ++kk) im[kk] = rl(gimg[kk]);
#pragma unroll
                for (int kk = 0; kk < RGB; ++kk)
                    if ((h >> kk) & 1) base ^= im[kk];
                const uint32_t ts = rl(gt);
                if (kg == KIND_CV || kg == KIND_CVDG)
                    elite64_pairs<NQ, W, true>(M, kg, base, im + RGB, ts, j);
                else
                    elite64_pairs<NQ, W, false>(M, kg, base, im + RGB, ts, j);
                wave_lds_fence();
            }
        }
        if (valid && !ok && !err) err = QE_DEVERR_DESC;
    }
    auto stored = [&](uint32_t r) -> uint32_t {      // stored row of logical row r
        uint32_t s = b;
#pragma unroll
        for (int p = 0; p < NQ; ++p)
            if ((r >> p) & 1) s ^= (uint32_t)(A >> (6 * p)) & 63u;
        return s;
    };
    // Eq. 11 (or the phase-insensitive form): the off-diagonal energy over
    // the lane's logical rows h, h + RG, ..., summed over the wavefronts of
    // the circuit in order; then the first wavefront reads the diagonal
    double off = 0.0;
    if (ok) {
        const uint32_t sh = stored((uint32_t)h);
#pragma unroll
        for (int m = 0; m < N / RG; ++m) {
            const uint32_t sr = sh ^ (stored((uint32_t)(m * RG)) ^ b);
            const double2 v = M[(sr << NQ) | (uint32_t)j];
            if (h + m * RG != j) off += v.x * v.x + v.y * v.y;
        }
    }
    off = wave_sum(off);
    if constexpr (W > 1) {
        if (lane == 0) red[circ][wv] = off;
        __syncthreads();
        off = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) off += red[circ][w];
    }
    if (wv != 0 || !valid) return;
    double dr = 0.0, di = 0.0;
    if (ok && lane < N) {
        const double2 v = M[(stored((uint32_t)lane) << NQ) | (uint32_t)lane];
        dr = v.x;
        di = v.y;
    }
    double fv, gv, dl;
    if (a.fit_mode == QE_FIT_PHASE_INSENSITIVE) {
        fitness_pi(off, N, &fv, &gv, &dl);
    } else {
        const double tr = wave_sum(dr), ti = wave_sum(di);
        const double am = sqrt(tr * tr + ti * ti);
        double er = 1.0, ei = 0.0;
        if (am > 0.0) { er = tr / am; ei = ti / am; }
        double D = 0.0;
        if (lane < N) { const double xr = dr - er, xi = di - ei; D = xr * xr + xi * xi; }
        dl = 0.5 * (off + wave_sum(D));
        double q = dl / (double)N;
        q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
        fv = 1.0 - sqrt(q);
    }
    if (lane == 0) {
        if (ok && !(fv == fv)) err = QE_DEVERR_NUMERIC;
        f64[ci] = ok ? fv : (double)__builtin_nan("");
        if (err) atomicOr(a.err, err);
    }
}

// Complex128 -> complex64 copy of the targets for the FP32 path.
__global__ void c128_to_c64_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) dst[idx] = (float)src[idx];
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_qeqea_init(const LoopArgs& a, hipStream_t s) {
    qeqea_init_kernel<<<blocks((size_t)a.I * a.S, 256), 256, 0, s>>>(a, (float)(1.0 / sqrt(3.0)));
    inst_best_init_kernel<<<blocks(a.I, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_ga_init(const LoopArgs& a, hipStream_t s) {
    if (a.inst_n) ga_init_mixed_kernel<<<a.I, 256, 0, s>>>(a);
    else ga_init_kernel<<<blocks((size_t)a.I * a.P * a.L, 256), 256, 0, s>>>(a);
    inst_best_init_kernel<<<blocks(a.I, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n > 0) fill_i32_kernel<<<blocks((size_t)n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_c128_to_c64(const double* src, float* dst, int64_t n_reals, hipStream_t s) {
    if (n_reals > 0) c128_to_c64_kernel<<<blocks((size_t)n_reals, 256), 256, 0, s>>>(src, dst, n_reals);
    return hipGetLastError();
}

hipError_t launch_gen_advance(uint64_t* g, uint64_t by, hipStream_t s) {
    gen_advance_kernel<<<1, 1, 0, s>>>(g, by);
    return hipGetLastError();
}

hipError_t launch_gen_set(uint64_t* g, uint64_t v, hipStream_t s) {
    gen_set_kernel<<<1, 1, 0, s>>>(g, v);
    return hipGetLastError();
}

hipError_t launch_qeqea_sample(const LoopArgs& a, uint64_t gen, uint32_t* slots, uint16_t* gates,
                               uint32_t* angles, hipStream_t s) {
    qeqea_sample_kernel<<<blocks((size_t)a.I * a.P * a.L, 256), 256, 0, s>>>(a, gen, slots, gates, angles);
    return hipGetLastError();
}

hipError_t launch_ga_copy(const LoopArgs& a, uint64_t gen, uint16_t* gates, hipStream_t s) {
    ga_copy_kernel<<<blocks((size_t)a.genes, 256), 256, 0, s>>>(a, gen, gates);
    return hipGetLastError();
}

template <bool SAMPLE>
static void launch_population(const LoopArgs& a, uint64_t gen, const uint16_t* gin, const uint32_t* ain,
                              uint32_t* sout, uint16_t* gout, uint32_t* aout, float* f, hipStream_t s,
                              bool decide = false) {
    const uint32_t total = (uint32_t)a.I * (uint32_t)a.P;
    const unsigned wb = blocks(total, 4);
    const Sched sc = schedule_for(a.n, a.L, a.lib == LIB_ISING ? SCHED_ISING : (SAMPLE ? SCHED_SAMPLED : SCHED_DISCRETE));
    // the LDS-staged kernels of widths 4 and 5 under the schedule (waves per
    // circuit; circuits per workgroup with one wavefront per circuit)
    auto lds45 = [&](auto nq, auto ising) {
        constexpr int NQ = decltype(nq)::value;
        constexpr bool IS = decltype(ising)::value;
        if constexpr (NQ == 5) {
            if (sc.waves == 2) {
                population_kernel<NQ, 2, SAMPLE, IS><<<total, 128, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide);
                return;
            }
        }
        if (sc.cpb == 1)
            population_kernel<NQ, 1, SAMPLE, IS, 1><<<total, 64, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide);
        else
            population_kernel<NQ, 1, SAMPLE, IS, 4><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide);
    };
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (a.lib == LIB_ISING) {
        // one wavefront per circuit below 4 wires, the LDS-staged layout above
        switch (a.n) {
            case 2: population_kernel<2, 0, SAMPLE, true><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
            case 3: population_kernel<3, 0, SAMPLE, true><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
            case 4: lds45(I4{}, T_{}); break;
            case 5: lds45(I5{}, T_{}); break;
            default: population_kernel<6, 4, SAMPLE, true><<<total, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        }
        return;
    }
    if (sc.lds && a.n >= 4) {
        switch (a.n) {
            case 4: lds45(I4{}, F_{}); break;
            case 5: lds45(I5{}, F_{}); break;
            default: population_kernel<6, 4, SAMPLE><<<total, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        }
        return;
    }
    switch (a.n) {
        case 1: population_kernel<1, 0, SAMPLE><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        case 2: population_kernel<2, 0, SAMPLE><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        case 3: population_kernel<3, 0, SAMPLE><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        case 4: population_kernel<4, 0, SAMPLE><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        case 5: population_kernel<5, 0, SAMPLE><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
        default: population_kernel<6, 0, SAMPLE><<<wb, 256, 0, s>>>(a, gen, gin, ain, sout, gout, aout, f, decide); break;
    }
}

hipError_t launch_eval_population(const LoopArgs& a, const uint16_t* gates, const uint32_t* angles,
                                  float* f, hipStream_t s) {
    launch_population<false>(a, 0, gates, angles, nullptr, nullptr, nullptr, f, s);
    return hipGetLastError();
}

hipError_t launch_ga_eval(const LoopArgs& a, uint64_t gen, float* f, hipStream_t s) {
    // the population of generation gen is genomes[gen & 1]; the parity is
    // resolved on the device for graph replays
    LoopArgs b = a;
    b.gen_ptr = nullptr;
    if (a.gen_ptr) return hipErrorInvalidValue;   // callers use launch_ga_copy + eval in graphs
    launch_population<false>(b, 0, a.genomes[gen & 1], nullptr, nullptr, nullptr, nullptr, f, s);
    return hipGetLastError();
}

hipError_t launch_qeqea_fused(const LoopArgs& a, uint64_t gen, uint32_t* slots, uint16_t* gates,
                              uint32_t* angles, float* f, bool decide, hipStream_t s) {
    launch_population<true>(a, gen, nullptr, nullptr, slots, gates, angles, f, s, decide);
    return hipGetLastError();
}

hipError_t launch_mutation_decisions(const LoopArgs& a, uint64_t gen, hipStream_t s) {
    mutation_decision_kernel<<<blocks((size_t)a.I * a.P, 256), 256, 0, s>>>(a, gen);
    return hipGetLastError();
}

hipError_t launch_scatter(const LoopArgs& a, uint64_t gen, const uint32_t* slots, const float* f,
                          hipStream_t s) {
    (void)gen;
    scatter_kernel<<<blocks((size_t)a.I * a.P * a.L, 256), 256, 0, s>>>(a, slots, f);
    return hipGetLastError();
}

hipError_t launch_dedup(const LoopArgs& a, uint64_t gen, hipStream_t s) {
    if (!a.dup) return hipSuccess;
    dedup_kernel<<<a.I, 256, (size_t)dedup_table((uint32_t)a.L * (uint32_t)a.P) * 4, s>>>(a, gen);
    return hipGetLastError();
}

hipError_t launch_qeqea_update(const LoopArgs& a, uint64_t gen, const uint32_t* slots,
                               const uint16_t* gates, const uint32_t* angles, const float* f,
                               hipStream_t s, bool shared, bool dedup_next) {
    if (a.P > UPD_MAX_P || ((shared || dedup_next) && !a.dup)) return hipErrorInvalidValue;
    const uint32_t nC = blocks((size_t)a.I * part_c_waves(a.P), UPD_BLOCK / 64);
    // part A: one workgroup per population over its shared entries, or one
    // thread per entry
    const uint32_t nA = shared ? (uint32_t)a.I : blocks((size_t)a.I * a.P * a.L, UPD_BLOCK);
    // part B: per instance, enough workgroups for the (mutated individual,
    // slot chunk) items up to four standard deviations above the binomial
    // mean (more items loop).  With many instances the grid holds far more
    // workgroups than the GPU runs at once and the total is close to its mean,
    // so the slack only adds workgroups that find nothing to do: then each
    // instance gets its mean and the busier ones loop.
    const double pm = (double)a.thr_pm / 4294967296.0;
    const bool many = pm * a.P * a.I * (((double)a.R * a.L + 255.0) / 256.0) > 8192.0;
    const int spl = many ? 4 : 1;
    const size_t chunks = ((size_t)a.R * a.L + 64 * spl - 1) / (64 * spl);
    const double expect = pm * a.P * chunks, sd = std::sqrt(a.P * pm * (1.0 - pm)) * chunks;
    const double slack = expect * a.I > 8192.0 ? 1.0 : 4.0 * sd + 8.0;
    // (each workgroup serves UPD_WPB items at once, one per wavefront)
    const uint32_t per_inst = (uint32_t)std::max<double>(
        1.0, std::ceil(std::min<double>(std::ceil(expect + slack), (double)a.P * chunks) / UPD_WPB));
    const uint32_t nB = per_inst * (uint32_t)a.I;
    // part D: one workgroup per population
    const uint32_t nD = dedup_next ? (uint32_t)a.I : 0u;
    size_t lds = ((size_t)a.P * sizeof(uint16_t) + 15) & ~(size_t)15;
    if (nD) lds = std::max(lds, (size_t)dedup_table((uint32_t)a.L * (uint32_t)a.P) * 4);
    const uint32_t a0 = (((nC + nB + 7u) & ~7u) + nD + 7u) & ~7u;
    if (many)
        qeqea_update_kernel<4><<<a0 + nA, UPD_BLOCK, lds, s>>>(a, gen, slots, gates, angles, f, nC, nB, nD,
                                                               per_inst, shared);
    else
        qeqea_update_kernel<1><<<a0 + nA, UPD_BLOCK, lds, s>>>(a, gen, slots, gates, angles, f, nC, nB, nD,
                                                               per_inst, shared);
    return hipGetLastError();
}

hipError_t launch_mutmask_clear(const LoopArgs& a, hipStream_t s) {
    const size_t n = (size_t)2 * a.I * a.MW;
    if (n) mutmask_clear_kernel<<<blocks(n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_state_gather(const LoopArgs& a, int which, void* dst, hipStream_t s) {
    const size_t n = (which == 1 || which == 4) ? (size_t)a.I * a.Q * 6 : (size_t)a.I * a.S;
    if (n) state_gather_kernel<<<blocks(n, 256), 256, 0, s>>>(a, which, dst);
    return hipGetLastError();
}

hipError_t launch_ga_update(const LoopArgs& a, uint64_t gen, const float* f, hipStream_t s) {
    ga_update_kernel<<<a.I, 256, 0, s>>>(a, gen, f);
    return hipGetLastError();
}

size_t elite_cand_keys(int I, int P) {
    return (size_t)I * (size_t)((P + ELITE_TILE - 1) / ELITE_TILE) * ELITE_MAX_TILE_K;
}

hipError_t launch_elite_select(const LoopArgs& a, const float* f, int k, int32_t* idx,
                               unsigned long long* cand, hipStream_t s) {
    auto np2 = [](int x) { int v = 1; while (v < x) v <<= 1; return v; };
    const int T = (a.P + ELITE_TILE - 1) / ELITE_TILE;
    if (T == 1 || k <= ELITE_MAX_TILE_K) {
        elite_select_kernel<ELITE_TILES><<<a.I * T, ELITE_TILE / 4, ELITE_TILE * 8, s>>>(a, f, k, T, cand,
                                                                                          idx);
        if (T > 1) {
            const int nk = std::max(ELITE_TILE, np2(T * k));
            elite_select_kernel<ELITE_MERGE><<<a.I, nk / 4, (size_t)nk * 8, s>>>(a, f, k, T, cand, idx);
        }
    } else {
        const int nk = std::max(ELITE_TILE, np2(a.P));
        elite_select_kernel<ELITE_WHOLE><<<a.I, nk / 4, (size_t)nk * 8, s>>>(a, f, k, T, nullptr, idx);
    }
    return hipGetLastError();
}

hipError_t launch_elite_eval(const LoopArgs& a, const uint16_t* gates, const uint32_t* angles, int k,
                             const int32_t* idx, double* f64, hipStream_t s) {
    // uniform widths 4 and 5 over a discrete library: one wavefront per circuit
    const unsigned nc = (unsigned)a.I * (unsigned)k;
    if (!a.inst_n && !angles && a.n == 5) {
        elite64_kernel<5, 2, 2><<<(nc + 1) / 2, 256, 0, s>>>(a, gates, k, idx, f64);
    } else if (!a.inst_n && !angles && a.n == 4) {
        elite64_kernel<4, 1, 4><<<(nc + 3) / 4, 256, 0, s>>>(a, gates, k, idx, f64);
    } else {
        elite_eval_kernel<<<nc, 256, generic_lds_bytes(a.n, sizeof(double)), s>>>(a, gates, angles, k, idx, f64);
    }
    return hipGetLastError();
}

}  // namespace qe
