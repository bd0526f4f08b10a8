// libqe C ABI: argument validation, context ownership, launches, graph
// capture of the generation loop, checkpoint / restore.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qe.h"
#include "qe_common.hpp"
#include "qe_internal.hpp"

using namespace qe;

namespace {

thread_local std::string g_last_error;

qe_status fail(qe_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

#define QE_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(QE_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// The device error word: a module global, so every device holds its own copy,
// zero from the moment the code object is loaded.  Its device address is
// resolved once per device (no allocation, no synchronisation, so calls that
// raise errors can be captured in graphs).
__device__ uint32_t g_dev_err_word;

std::mutex g_mu;
std::map<int, uint32_t*> g_err_words;

qe_status device_error_word(uint32_t** out) {
    int dev = 0;
    QE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_err_words.find(dev);
    if (it != g_err_words.end()) { *out = it->second; return QE_OK; }
    uint32_t* p = nullptr;
    QE_HIP(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(g_dev_err_word)));
    g_err_words[dev] = p;
    *out = p;
    return QE_OK;
}

// Scratch of the allocation-free evaluation (qe_eval_fitness_noalloc): the
// item table and cost order of a mixed-width batch of at most
// QE_NOALLOC_MAX_CIRCUITS circuits.  A module global: each device holds its
// own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is only a stand-in
// for the symbol): it uses the device address that hipGetSymbolAddress
// gives, resolved once per device on the entry point's first call there.
// Nothing in it must start at zero: the sort kernel writes every entry the
// evaluation kernel reads.  All calls on one device share it.
static __device__ __align__(256) int32_t scratch[MIX_WORK_META + QE_NOALLOC_MAX_CIRCUITS];
std::map<int, int32_t*> g_scratch;

qe_status noalloc_scratch(int32_t** out) {
    int dev = 0;
    QE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) { *out = it->second; return QE_OK; }
    int32_t* p = nullptr;
    QE_HIP(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(QE_ERR_DEVICE, "hipGetSymbolAddress gave no address for the scratch array");
    g_scratch[dev] = p;
    *out = p;
    return QE_OK;
}

// Schedule of the FP32 path per width, length class (0: L < 32, 1: L >= 32)
// and library class (SCHED_*): the LDS-staged kernel or the register-resident
// one, the LDS kernel's wavefronts per circuit and (one wavefront per
// circuit) circuits per workgroup of the population kernels.  Defaults from
// MI355X measurements; the tuning table written by
// paper_1809_11134_amd/tune.py replaces them, and
// QE_SCHEDULE="n:lds[:waves[:cpb]],..." overrides every class of a width.
Sched g_sched[MAX_QUBITS + 1][2][SCHED_CLASSES];
std::once_flag g_sched_once;

// MFMA paths: fewest non-identity gates of a fused block, per width and
// length class (1: every group is fused); table lines "mfma n lclass v"
int g_mfma_min[MAX_QUBITS + 1][2];
constexpr int MFMA_MIN_BLOCK_MAX = 65;       // above the 64 gates of a chunk: never fuse

void default_schedules() {
    for (int n = 0; n <= MAX_QUBITS; ++n)
        for (int l = 0; l < 2; ++l)
            for (int c = 0; c < SCHED_CLASSES; ++c)
                g_sched[n][l][c] = n <= 3 ? Sched{0, 1, 4} : (n == 6 ? Sched{1, 4, 1} : Sched{1, 1, 4});
    for (int n = 0; n <= MAX_QUBITS; ++n) g_mfma_min[n][0] = g_mfma_min[n][1] = 1;
}

void set_classes(int n, int l, const Sched& v) {
    for (int c = 0; c < SCHED_CLASSES; ++c) g_sched[n][l][c] = v;
}

// wavefronts per circuit the LDS kernels are built for, per width
bool waves_ok(int n, int w) {
    if (n <= 3) return w == 1;
    if (n == 4) return w == 1;
    if (n == 5) return w == 1 || w == 2;
    return w == 4;
}

bool sched_ok(int n, int lds, int w, int cpb) {
    return n >= 1 && n <= MAX_QUBITS && (lds == 0 || lds == 1) && waves_ok(n, w) && (cpb == 1 || cpb == 4);
}

// Tuning table lines: "n lclass lib lds waves cpb" (one length and library
// class), "n lclass lds waves cpb" (one length class, every library class),
// or "n lds" (every class, default waves and cpb); '#' starts a comment.
// Path: $QE_TUNE_TABLE, else tune_mi355x.txt next to libqe.so.
void load_tune_table() {
    std::string path;
    if (const char* e = std::getenv("QE_TUNE_TABLE")) {
        path = e;
    } else {
        Dl_info info;
        if (dladdr((void*)&load_tune_table, &info) && info.dli_fname) {
            std::string so(info.dli_fname);
            const size_t slash = so.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune_mi355x.txt";
        }
    }
    FILE* fh = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!fh) return;
    char line[256];
    while (std::fgets(line, sizeof line, fh)) {
        if (line[0] == '#') continue;
        if (char* c = std::strchr(line, '#')) *c = 0;
        {
            int n = 0, l = 0, v = 0;
            if (std::sscanf(line, " mfma %d %d %d", &n, &l, &v) == 3) {
                if (n >= 1 && n <= MAX_QUBITS && (l == 0 || l == 1) && v >= 1 && v <= MFMA_MIN_BLOCK_MAX)
                    g_mfma_min[n][l] = v;
                continue;
            }
        }
        int n = 0, x1 = 0, x2 = 0, x3 = 0, x4 = 0, x5 = 0;
        const int got = std::sscanf(line, "%d %d %d %d %d %d", &n, &x1, &x2, &x3, &x4, &x5);
        if (got == 6 && (x1 == 0 || x1 == 1) && x2 >= 0 && x2 < SCHED_CLASSES && sched_ok(n, x3, x4, x5)) {
            g_sched[n][x1][x2] = Sched{x3, x4, x5};
        } else if (got == 5 && (x1 == 0 || x1 == 1) && sched_ok(n, x2, x3, x4)) {
            set_classes(n, x1, Sched{x2, x3, x4});
        } else if (got == 2 && n >= 1 && n <= MAX_QUBITS) {
            for (int l = 0; l < 2; ++l)
                for (int c = 0; c < SCHED_CLASSES; ++c) g_sched[n][l][c].lds = x1 ? 1 : 0;
        }
    }
    std::fclose(fh);
}

void load_schedule_env() {
    default_schedules();
    load_tune_table();
    const char* s = std::getenv("QE_SCHEDULE");
    if (!s) return;
    std::string str(s);
    size_t pos = 0;
    while (pos < str.size()) {
        size_t comma = str.find(',', pos);
        std::string item = str.substr(pos, comma == std::string::npos ? std::string::npos : comma - pos);
        int n = 0, l = 0, w = 0, c = 0;
        const int got = std::sscanf(item.c_str(), "%d:%d:%d:%d", &n, &l, &w, &c);
        if (got >= 2 && n >= 1 && n <= MAX_QUBITS) {
            for (int k = 0; k < 2; ++k)
                for (int cl = 0; cl < SCHED_CLASSES; ++cl) {
                    Sched v = g_sched[n][k][cl];
                    v.lds = l ? 1 : 0;
                    if (got >= 3) v.waves = w;
                    if (got >= 4) v.cpb = c;
                    if (sched_ok(n, v.lds, v.waves, v.cpb)) g_sched[n][k][cl] = v;
                }
        }
        if (comma == std::string::npos) break;
        pos = comma + 1;
    }
}

uint64_t prob_threshold(double p) {
    if (!(p > 0)) return 0;
    if (p >= 1) return (uint64_t)1 << 32;
    return (uint64_t)std::floor(p * 4294967296.0);
}

qe_status to_args(const qe_batch* b, BatchArgs* a, bool need_targets) {
    if (!b) return fail(QE_ERR_INVALID, "batch is NULL");
    if (b->num_circuits < 0) return fail(QE_ERR_INVALID, "num_circuits < 0");
    if (b->uniform_n < 0 || b->uniform_n > MAX_QUBITS)
        return fail(QE_ERR_INVALID, "uniform_n must be 0 (mixed) or 1..6");
    if (b->uniform_n == 0 && b->num_circuits > 0 && !b->n_qubits_dev)
        return fail(QE_ERR_INVALID, "mixed widths need n_qubits_dev");
    if (b->uniform_L < 0) return fail(QE_ERR_INVALID, "uniform_L < 0");
    if (b->uniform_L == 0 && b->num_circuits > 0 && !b->gate_offsets_dev)
        return fail(QE_ERR_INVALID, "uneven lengths need gate_offsets_dev");
    if (b->num_gates < 0) return fail(QE_ERR_INVALID, "num_gates < 0");
    if (b->uniform_L > 0 && (int64_t)b->num_circuits * b->uniform_L > b->num_gates)
        return fail(QE_ERR_INVALID, "num_circuits * uniform_L exceeds num_gates");
    if (b->num_gates > 0 && !b->gates_dev) return fail(QE_ERR_INVALID, "gates_dev is NULL");
    if (b->fitness_mode != QE_FIT_EQ11 && b->fitness_mode != QE_FIT_PHASE_INSENSITIVE)
        return fail(QE_ERR_INVALID, "unknown fitness_mode");
    if (need_targets) {
        if (b->target_stride < 0 && b->num_circuits > 0 && !b->target_offsets_dev)
            return fail(QE_ERR_INVALID, "target_stride < 0 needs target_offsets_dev");
        if (b->num_circuits > 0 && !b->targets_dev) return fail(QE_ERR_INVALID, "targets_dev is NULL");
        if (b->num_target_elems < 0) return fail(QE_ERR_INVALID, "num_target_elems < 0");
        if (b->uniform_n > 0 && b->target_stride >= 0 && b->num_circuits > 0) {
            const int64_t NN = (int64_t)1 << (2 * b->uniform_n);
            if ((int64_t)(b->num_circuits - 1) * b->target_stride + NN > b->num_target_elems)
                return fail(QE_ERR_INVALID, "targets buffer too small for the stride");
        }
    }
    a->B = b->num_circuits;
    a->uniform_n = b->uniform_n;
    a->nq = b->n_qubits_dev;
    a->uniform_L = b->uniform_L;
    a->goff = b->gate_offsets_dev;
    a->gates = b->gates_dev;
    a->num_gates = b->num_gates;
    a->tstride = b->target_stride;
    a->toff = b->target_offsets_dev;
    a->targets = b->targets_dev;
    a->num_telems = b->num_target_elems;
    a->mode = b->fitness_mode;
    a->mix_w5 = schedule_for(5, 32, b->angles_dev ? SCHED_ISING : SCHED_DISCRETE).waves;
    a->angles = b->angles_dev;
    return device_error_word(&a->err);
}

}  // namespace

namespace qe {
Sched schedule_for(int n, int L, int lib_class) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS) return Sched{0, 1, 4};
    if (lib_class < 0 || lib_class >= SCHED_CLASSES) lib_class = SCHED_DISCRETE;
    return g_sched[n][L >= 32 ? 1 : 0][lib_class];
}
bool schedule_lds(int n) { return schedule_for(n, 32).lds != 0; }
int mfma_min_block(int n, int L) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS) return 1;
    return g_mfma_min[n][L >= 32 ? 1 : 0];
}
}  // namespace qe

// ====================================================================== ctx
struct qe_ctx {
    qe_problem prob;
    int device = 0;
    LoopArgs la{};
    int N = 0;
    size_t S = 0, Q = 0;          // per instance
    bool targets_set = false;
    // ctx-owned device buffers
    std::vector<void*> owned;
    uint16_t* gates = nullptr;    // [I*P*L]
    uint32_t* angles = nullptr;   // [I*P*L] (Ising library)
    float* f = nullptr;           // [I*P]
    uint64_t* d_gen = nullptr;
    unsigned long long* elite_cand = nullptr;   // candidates of the tiled elite selection
    hipStream_t capture_stream = nullptr;
    std::map<std::pair<int, float*>, hipGraphExec_t> graphs;
    hipGraph_t last_graph = nullptr;
    // the generation whose mutation decisions may be appended to the lists
    // without emptying them first (the one after the last decided)
    uint64_t next_decision_gen = 0;
    // the generation of the last qe_sample_eval (its segment keys and mutation
    // decisions are in place for qe_update), -1 when another call came since
    int64_t fused_gen = -1;
    // QEQEA with the shared-slot search: the generation whose slot words each
    // of the two buffers holds (buffer g & 1 for generation g; -1 none).  The
    // words depend on the seed and the generation only, so they stay valid
    // until the buffer is written for another generation.
    int64_t words_gen[2] = {-1, -1};
    // mixed GA populations (qe_create_mixed): per population width, genome
    // length and target offset (host copies), genes per genome buffer,
    // complex elements of the targets; per circuit width, gate offsets and
    // target offsets for the evaluation; the cost order of the circuits
    // (fixed by widths and lengths, computed once) and a workspace that
    // qe_eval_fitness may use for other mixed batches
    bool mixed = false;
    std::vector<int32_t> inst_n, inst_L;
    std::vector<int64_t> inst_toff;
    int64_t genes = 0;
    int64_t target_elems = 0;
    int8_t* circ_n = nullptr;
    int32_t* circ_goff = nullptr;
    int64_t* circ_toff = nullptr;
    int32_t* mix_order = nullptr;
    int32_t* mix_eval_work = nullptr;
    size_t mix_work_bytes = 0;
    uint32_t* check_word = nullptr;   // flags of the phase-insensitive target check
    int32_t mix_w5 = 1;               // the schedule the mixed order was computed for
};

namespace {

template <typename T>
qe_status ctx_alloc(qe_ctx* c, T** p, size_t elems) {
    void* q = nullptr;
    if (elems == 0) elems = 1;
    hipError_t e = hipMalloc(&q, elems * sizeof(T));
    if (e != hipSuccess) return fail(QE_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->owned.push_back(q);
    *p = static_cast<T*>(q);
    return QE_OK;
}

// Releases everything the context owns (best effort: a failing release
// cannot be undone, and the remaining ones still run).
void free_ctx(qe_ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (void* p : c->owned) (void)hipFree(p);
    delete c;
}

#define QE_TRY(x)                        \
    do {                                 \
        qe_status s_ = (x);              \
        if (s_ != QE_OK) return s_;      \
    } while (0)

bool is_ising(const qe_ctx* c) { return c->prob.library == QE_LIB_ISING; }

qe_status check_ctx(qe_ctx* c, bool need_targets) {
    if (!c) return fail(QE_ERR_INVALID, "ctx is NULL");
    if (need_targets && !c->targets_set) return fail(QE_ERR_STATE, "qe_set_targets has not been called");
    return QE_OK;
}

// sample + eval + update of one generation (gen is relative to la.gen_ptr
// when graph-captured).
// Before the mutation decisions of generation `gen` (first of `count`
// consecutive ones): the decision masks are cleared unless the previous
// decisions were those of gen - 1, whose kernels cleared the mask of gen's
// parity.
qe_status prepare_decisions(qe_ctx* c, uint64_t gen, uint64_t count, hipStream_t s) {
    if (c->prob.algorithm != QE_ALG_QEQEA) return QE_OK;
    if (gen != c->next_decision_gen) QE_HIP(launch_mutmask_clear(c->la, s));
    c->next_decision_gen = gen + count;
    return QE_OK;
}

// The evaluation batch of a mixed context's I*P circuits (genomes in `gates`,
// laid out as the genome buffers).
BatchArgs mixed_batch(const qe_ctx* c, const uint16_t* gates) {
    BatchArgs b{};
    b.B = c->prob.n_instances * c->prob.size_of_population;
    b.uniform_n = 0;
    b.nq = c->circ_n;
    b.uniform_L = 0;
    b.goff = c->circ_goff;
    b.gates = gates;
    b.num_gates = c->genes;
    b.tstride = -1;
    b.toff = c->circ_toff;
    b.targets = c->la.target32;
    b.num_telems = c->target_elems;
    b.mode = c->prob.fitness_mode;
    b.mix_w5 = c->mix_w5;
    b.angles = nullptr;
    b.err = c->la.err;
    return b;
}

void note_words(qe_ctx* c, uint64_t gen) {
    if (c->la.dup) c->words_gen[gen & 1] = (int64_t)gen;
}

// The shared-slot search of generation gen, unless its words are in place.
qe_status ensure_words(qe_ctx* c, uint64_t gen, hipStream_t s) {
    if (!c->la.dup || c->words_gen[gen & 1] == (int64_t)gen) return QE_OK;
    QE_HIP(launch_dedup(c->la, gen, s));
    note_words(c, gen);
    return QE_OK;
}

// One generation.  QEQEA: the slot words of the generation must be in place
// (ensure_words, or the update of the generation before it); the update runs
// the next generation's search.
qe_status enqueue_generation(qe_ctx* c, const LoopArgs& a, uint64_t gen, float* f, hipStream_t s) {
    if (c->prob.algorithm == QE_ALG_QEQEA) {
        // without slot words the update draws each entry's slot again; with
        // them it walks the search's list of shared entries (the fused kernel
        // committed the others)
        QE_HIP(launch_qeqea_fused(a, gen, nullptr, c->gates, c->angles, f, true, s));
        QE_HIP(launch_qeqea_update(a, gen, nullptr, c->gates, c->angles, f, s, a.dup != nullptr,
                                   a.dup != nullptr));
    } else {
        QE_HIP(launch_ga_copy(a, gen, c->gates, s));
        if (c->mixed) QE_HIP(launch_mix_eval(mixed_batch(c, c->gates), c->mix_order, f, nullptr, nullptr, s));
        else QE_HIP(launch_eval_population(a, c->gates, nullptr, f, s));
        QE_HIP(launch_ga_update(a, gen, f, s));
    }
    return QE_OK;
}

}  // namespace

extern "C" {

const char* qe_last_error(void) { return g_last_error.c_str(); }
const char* qe_version(void) { return "libqe 0.1 (gfx950)"; }

int32_t qe_lib_size(int32_t library, int32_t n) {
    if ((library != 0 && library != 1) || n < 1 || n > MAX_QUBITS) return -1;
    return lib_size(library, n);
}

qe_status qe_lib_table(int32_t library, int32_t n, uint16_t* table_host) {
    if ((library != 0 && library != 1) || n < 1 || n > MAX_QUBITS || !table_host)
        return fail(QE_ERR_INVALID, "bad library, width or NULL table");
    for (int i = 0; i < lib_size(library, n); ++i) table_host[i] = lib_desc(library, n, i);
    return QE_OK;
}

qe_status qe_set_schedule(int32_t n, int32_t lds) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS) return fail(QE_ERR_INVALID, "width must be 1..6");
    for (int l = 0; l < 2; ++l)
        for (int c = 0; c < SCHED_CLASSES; ++c) g_sched[n][l][c].lds = lds ? 1 : 0;
    return QE_OK;
}

qe_status qe_get_schedule(int32_t n, int32_t* lds) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS || !lds) return fail(QE_ERR_INVALID, "width must be 1..6");
    *lds = g_sched[n][1][SCHED_DISCRETE].lds;
    return QE_OK;
}

qe_status qe_set_schedule_ex(int32_t n, int32_t lclass, int32_t lds, int32_t waves, int32_t cpb) {
    std::call_once(g_sched_once, load_schedule_env);
    if (lclass != 0 && lclass != 1) return fail(QE_ERR_INVALID, "lclass must be 0 (L < 32) or 1 (L >= 32)");
    if (!sched_ok(n, lds, waves, cpb))
        return fail(QE_ERR_INVALID, "no such schedule: lds 0/1; waves 1 (n <= 5), 2 (n = 5) or 4 (n = 6); cpb 1 or 4");
    set_classes(n, lclass, Sched{lds, waves, cpb});
    return QE_OK;
}

qe_status qe_get_schedule_ex(int32_t n, int32_t lclass, int32_t* lds, int32_t* waves, int32_t* cpb) {
    return qe_get_schedule_lib(n, lclass, QE_SCHED_DISCRETE, lds, waves, cpb);
}

qe_status qe_set_mfma_min_block(int32_t n, int32_t lclass, int32_t min_block) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS || (lclass != 0 && lclass != 1) || min_block < 1 ||
        min_block > MFMA_MIN_BLOCK_MAX)
        return fail(QE_ERR_INVALID, "width 1..6, lclass 0 or 1, min_block 1..65");
    g_mfma_min[n][lclass] = min_block;
    return QE_OK;
}

qe_status qe_get_mfma_min_block(int32_t n, int32_t lclass, int32_t* min_block) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS || (lclass != 0 && lclass != 1) || !min_block)
        return fail(QE_ERR_INVALID, "width 1..6, lclass 0 or 1, non-NULL output");
    *min_block = g_mfma_min[n][lclass];
    return QE_OK;
}

qe_status qe_set_schedule_lib(int32_t n, int32_t lclass, int32_t lib_class, int32_t lds, int32_t waves,
                              int32_t cpb) {
    std::call_once(g_sched_once, load_schedule_env);
    if (lclass != 0 && lclass != 1) return fail(QE_ERR_INVALID, "lclass must be 0 (L < 32) or 1 (L >= 32)");
    if (lib_class < 0 || lib_class >= SCHED_CLASSES)
        return fail(QE_ERR_INVALID, "lib_class must be QE_SCHED_DISCRETE, QE_SCHED_SAMPLED or QE_SCHED_ISING");
    if (!sched_ok(n, lds, waves, cpb))
        return fail(QE_ERR_INVALID, "no such schedule: lds 0/1; waves 1 (n <= 5), 2 (n = 5) or 4 (n = 6); cpb 1 or 4");
    g_sched[n][lclass][lib_class] = Sched{lds, waves, cpb};
    return QE_OK;
}

qe_status qe_get_schedule_lib(int32_t n, int32_t lclass, int32_t lib_class, int32_t* lds, int32_t* waves,
                              int32_t* cpb) {
    std::call_once(g_sched_once, load_schedule_env);
    if (n < 1 || n > MAX_QUBITS || (lclass != 0 && lclass != 1) || lib_class < 0 ||
        lib_class >= SCHED_CLASSES || !lds || !waves || !cpb)
        return fail(QE_ERR_INVALID, "width 1..6, lclass 0 or 1, lib_class 0..2, non-NULL outputs");
    const Sched v = g_sched[n][lclass][lib_class];
    *lds = v.lds;
    *waves = v.waves;
    *cpb = v.cpb;
    return QE_OK;
}

// ------------------------------------------------------------------- eval
size_t qe_eval_workspace_bytes(int32_t num_circuits) {
    return num_circuits < 0 ? 0 : ((size_t)MIX_WORK_META + (size_t)num_circuits) * sizeof(int32_t);
}

}  // extern "C"

namespace {

// Shared by the evaluation entry points: `work` (MIX_WORK_META + B int32 of
// device memory, or NULL) holds the order and item table of the cost-sorted
// single launch of a mixed-width FP32 batch; without it such a batch runs
// as one filtered launch per width.
qe_status eval_fitness_impl(const qe_batch* batch, int32_t path, float* f_dev, float* g_dev,
                            float* delta_dev, int32_t* work, size_t work_bytes, void* stream) {
    BatchArgs a;
    QE_TRY(to_args(batch, &a, true));
    if (path < QE_PATH_FP32 || path > QE_PATH_DENSE) return fail(QE_ERR_INVALID, "unknown path");
    if (a.B > 0 && !f_dev) return fail(QE_ERR_INVALID, "f_dev is NULL");
    if (a.angles && path != QE_PATH_FP32 && path != QE_PATH_FP32_LDS && path != QE_PATH_DENSE)
        return fail(QE_ERR_UNSUPPORTED,
                    "angled (Ising) batches run on QE_PATH_FP32 / QE_PATH_FP32_LDS / QE_PATH_DENSE");
    if (path >= QE_PATH_MFMA_BF16 && path != QE_PATH_DENSE && a.uniform_n != 5 && a.uniform_n != 6)
        return fail(QE_ERR_UNSUPPORTED, "MFMA paths need a uniform width of 5 or 6");
    if (work && work_bytes < qe_eval_workspace_bytes(a.B))
        return fail(QE_ERR_INVALID, "workspace smaller than qe_eval_workspace_bytes(num_circuits)");
    const hipStream_t s = (hipStream_t)stream;
    if (path == QE_PATH_DENSE) {
        QE_HIP(launch_eval_dense(a, f_dev, g_dev, delta_dev, s));
    } else if (path >= QE_PATH_MFMA_BF16) {
        const bool fp16 = path == QE_PATH_MFMA_FP16 || path == QE_PATH_MFMA_FP16_RAW;
        const bool renorm = path == QE_PATH_MFMA_BF16 || path == QE_PATH_MFMA_FP16;
        QE_HIP(launch_eval_mfma(a, fp16, renorm, f_dev, g_dev, delta_dev, s));
    } else {
        if (a.uniform_n != 0 || path != QE_PATH_FP32) work = nullptr;
        QE_HIP(launch_eval_fp32(a, path, f_dev, g_dev, delta_dev, work, s));
    }
    QE_HIP(launch_target_check(a, false, f_dev, g_dev, delta_dev, s));
    return QE_OK;
}

}  // namespace

extern "C" {

qe_status qe_eval_fitness(qe_ctx* ctx, const qe_batch* batch, int32_t path, float* f_dev,
                          float* g_dev, float* delta_dev, void* stream) {
    // a mixed-width context lends its workspace when the batch fits it
    int32_t* work = nullptr;
    size_t bytes = 0;
    if (ctx && ctx->mix_eval_work && batch && batch->num_circuits >= 0 &&
        qe_eval_workspace_bytes(batch->num_circuits) <= ctx->mix_work_bytes) {
        work = ctx->mix_eval_work;
        bytes = ctx->mix_work_bytes;
    }
    return eval_fitness_impl(batch, path, f_dev, g_dev, delta_dev, work, bytes, stream);
}

qe_status qe_eval_fitness_noalloc(const qe_batch* batch, int32_t path, float* f_dev, float* g_dev,
                                  float* delta_dev, void* stream) {
    if (batch && batch->uniform_n == 0 && path == QE_PATH_FP32 && batch->num_circuits > QE_NOALLOC_MAX_CIRCUITS)
        return fail(QE_ERR_INVALID, "qe_eval_fitness_noalloc: a mixed-width batch of more than "
                                    "QE_NOALLOC_MAX_CIRCUITS (" + std::to_string(QE_NOALLOC_MAX_CIRCUITS) +
                                    ") circuits");
    int32_t* work = nullptr;
    QE_TRY(noalloc_scratch(&work));
    return eval_fitness_impl(batch, path, f_dev, g_dev, delta_dev, work,
                             ((size_t)MIX_WORK_META + QE_NOALLOC_MAX_CIRCUITS) * sizeof(int32_t), stream);
}

qe_status qe_eval_fitness_ws(const qe_batch* batch, int32_t path, float* f_dev, float* g_dev,
                             float* delta_dev, void* workspace_dev, size_t workspace_bytes,
                             void* stream) {
    if (!workspace_dev) return fail(QE_ERR_INVALID, "workspace_dev is NULL");
    return eval_fitness_impl(batch, path, f_dev, g_dev, delta_dev, (int32_t*)workspace_dev,
                             workspace_bytes, stream);
}

qe_status qe_eval_fitness_fp64(const qe_batch* batch, double* f_dev, double* g_dev,
                               double* delta_dev, void* stream) {
    BatchArgs a;
    QE_TRY(to_args(batch, &a, true));
    if (a.B > 0 && !f_dev) return fail(QE_ERR_INVALID, "f_dev is NULL");
    QE_HIP(launch_eval_lds(a, true, f_dev, g_dev, delta_dev, (hipStream_t)stream));
    QE_HIP(launch_target_check(a, true, f_dev, g_dev, delta_dev, (hipStream_t)stream));
    return QE_OK;
}

qe_status qe_build_unitary(const qe_batch* batch, int32_t precision, void* out_dev,
                           int64_t out_elems, void* stream) {
    BatchArgs a;
    QE_TRY(to_args(batch, &a, false));
    if (a.uniform_n < 1) return fail(QE_ERR_INVALID, "qe_build_unitary needs uniform_n");
    if (precision != 0 && precision != 1) return fail(QE_ERR_INVALID, "precision must be 0 or 1");
    const int64_t need = (int64_t)a.B << (2 * a.uniform_n);
    if (out_elems < need) return fail(QE_ERR_INVALID, "out_elems too small");
    if (a.B > 0 && !out_dev) return fail(QE_ERR_INVALID, "out_dev is NULL");
    QE_HIP(launch_unitary(a, precision == 1, out_dev, (hipStream_t)stream));
    return QE_OK;
}

qe_status qe_device_errors(int32_t* flags_host) {
    if (!flags_host) return fail(QE_ERR_INVALID, "flags_host is NULL");
    uint32_t* w = nullptr;
    QE_TRY(device_error_word(&w));
    QE_HIP(hipDeviceSynchronize());
    uint32_t v = 0;
    QE_HIP(hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost));
    QE_HIP(hipMemset(w, 0, sizeof(uint32_t)));
    QE_HIP(hipDeviceSynchronize());
    *flags_host = (int32_t)v;
    return QE_OK;
}

// ------------------------------------------------------------------ context
}  // extern "C"

namespace {

// qe_create, and qe_create_mixed when inst_n / inst_L (host, I entries) are
// given: then every population has its own width and genome length, and
// the problem's n_qubits and size_of_individual are replaced by the maxima.
qe_status create_impl(const qe_problem* p_in, const int32_t* inst_n, const int32_t* inst_L, qe_ctx** out) {
    if (!p_in || !out) return fail(QE_ERR_INVALID, "NULL argument");
    *out = nullptr;
    qe_problem pm = *p_in;
    const qe_problem* p = &pm;
    const bool mixed = inst_n != nullptr;
    int64_t genes_per_ind = 0, target_elems = 0;
    if (mixed) {
        if (!inst_L) return fail(QE_ERR_INVALID, "inst_L is NULL");
        if (p->algorithm != QE_ALG_GA) return fail(QE_ERR_UNSUPPORTED, "mixed widths and lengths: GA only");
        if (p->library != QE_LIB_NCV && p->library != QE_LIB_HT_NCV)
            return fail(QE_ERR_UNSUPPORTED, "mixed populations take the discrete libraries");
        if (p->n_instances < 1 || p->n_instances > (1 << 20)) return fail(QE_ERR_INVALID, "n_instances must be 1..2^20");
        int nmax = 1, lmax = 1;
        for (int i = 0; i < p->n_instances; ++i) {
            if (inst_n[i] < 1 || inst_n[i] > MAX_QUBITS) return fail(QE_ERR_INVALID, "every width must be 1..6");
            if (inst_L[i] < 1 || inst_L[i] > 1024) return fail(QE_ERR_INVALID, "every genome length must be 1..1024");
            nmax = std::max(nmax, (int)inst_n[i]);
            lmax = std::max(lmax, (int)inst_L[i]);
            genes_per_ind += inst_L[i];
            target_elems += (int64_t)1 << (2 * inst_n[i]);
        }
        pm.n_qubits = nmax;
        pm.size_of_individual = lmax;
    }
    const int n = p->n_qubits;
    if (p->library != QE_LIB_NCV && p->library != QE_LIB_HT_NCV && p->library != QE_LIB_ISING)
        return fail(QE_ERR_INVALID, "unknown library");
    if (p->algorithm != QE_ALG_QEQEA && p->algorithm != QE_ALG_GA) return fail(QE_ERR_INVALID, "unknown algorithm");
    if (n < 1 || n > MAX_QUBITS) return fail(QE_ERR_INVALID, "n_qubits must be 1..6");
    if (p->algorithm == QE_ALG_QEQEA && n < 2) return fail(QE_ERR_INVALID, "QEQEA needs n_qubits >= 2");
    if (p->algorithm == QE_ALG_QEQEA && p->library == QE_LIB_HT_NCV)
        return fail(QE_ERR_UNSUPPORTED, "QEQEA decodes to {I, NOT, CNOT, CV, CV+} or the Ising library");
    if (p->algorithm == QE_ALG_GA && p->library == QE_LIB_ISING)
        return fail(QE_ERR_UNSUPPORTED, "the GA genome holds no angles: discrete libraries only");
    if (p->size_of_individual < 1 || p->size_of_individual > 1024) return fail(QE_ERR_INVALID, "L must be 1..1024");
    if (p->size_of_population < 1 || p->size_of_population > 65536) return fail(QE_ERR_INVALID, "P must be 1..65536");
    if (p->algorithm == QE_ALG_GA && p->size_of_population > 4096) return fail(QE_ERR_INVALID, "GA needs P <= 4096");
    if (p->algorithm == QE_ALG_QEQEA && p->size_of_population > 16384)
        return fail(QE_ERR_INVALID, "QEQEA needs P <= 16384");
    if (p->n_instances < 1) return fail(QE_ERR_INVALID, "n_instances must be >= 1");
    const double pi2 = 2.0 * 3.14159265358979323846;
    if (!(p->prob_mutation >= 0 && p->prob_mutation <= 1)) return fail(QE_ERR_INVALID, "prob_mutation must be in [0,1]");
    if (!(p->mutation_range >= 0 && p->mutation_range < pi2)) return fail(QE_ERR_INVALID, "mutation_range must be in [0, 2 pi)");
    if (!(p->ga_crossover_prob >= 0 && p->ga_crossover_prob <= 1)) return fail(QE_ERR_INVALID, "ga_crossover_prob must be in [0,1]");
    if (!(p->ga_gene_mutation_prob >= 0 && p->ga_gene_mutation_prob <= 1)) return fail(QE_ERR_INVALID, "ga_gene_mutation_prob must be in [0,1]");
    if (p->fitness_mode != QE_FIT_EQ11 && p->fitness_mode != QE_FIT_PHASE_INSENSITIVE)
        return fail(QE_ERR_INVALID, "unknown fitness_mode");
    const size_t L = p->size_of_individual, P = p->size_of_population, I = p->n_instances;
    const size_t R = (size_t)regions(n, p->library);
    const size_t S = R * L * P, Q = (size_t)n * L * P;
    if ((uint64_t)S >= (1ull << 32) || I * P * L >= (1ull << 32))
        return fail(QE_ERR_INVALID, "encoding too large (slot indices are 32-bit)");
    if (I > (1u << 31) / P) return fail(QE_ERR_INVALID, "too many instances");
    const int64_t genes = mixed ? genes_per_ind * (int64_t)P : (int64_t)(I * P * L);
    if (!mixed) target_elems = (int64_t)I << (2 * n);

    qe_ctx* c = new qe_ctx();
    // stored field by field over zeroed bytes, so that checkpoint headers
    // hold no stray padding
    std::memset(&c->prob, 0, sizeof(c->prob));
    c->prob.n_qubits = p->n_qubits;
    c->prob.library = p->library;
    c->prob.algorithm = p->algorithm;
    c->prob.size_of_individual = p->size_of_individual;
    c->prob.size_of_population = p->size_of_population;
    c->prob.n_instances = p->n_instances;
    c->prob.prob_mutation = p->prob_mutation;
    c->prob.mutation_range = p->mutation_range;
    c->prob.ga_crossover_prob = p->ga_crossover_prob;
    c->prob.ga_gene_mutation_prob = p->ga_gene_mutation_prob;
    c->prob.seed = p->seed;
    c->prob.fitness_mode = p->fitness_mode;
    if (hipGetDevice(&c->device) != hipSuccess) { free_ctx(c); return fail(QE_ERR_DEVICE, "hipGetDevice"); }
    c->N = 1 << n;
    c->S = S;
    c->Q = Q;
    LoopArgs& a = c->la;
    a.n = n; a.lib = p->library; a.L = (int)L; a.P = (int)P; a.I = (int)I;
    a.seed = p->seed;
    a.fit_mode = p->fitness_mode;
    a.thr_pm = prob_threshold((double)p->prob_mutation);
    a.thr_pc = prob_threshold((double)p->ga_crossover_prob);
    a.thr_pg = prob_threshold((double)p->ga_gene_mutation_prob);
    a.r32 = (float)((double)p->mutation_range / pi2 * 4294967296.0);
    a.R = (uint32_t)R;
    a.S = (uint32_t)S;
    a.Q = (uint32_t)Q;
    a.genes = genes;
    c->genes = genes;
    c->target_elems = target_elems;
    c->mixed = mixed;
    qe_status st = QE_OK;
#define ALLOC(ptr, n_) if (st == QE_OK) st = ctx_alloc(c, &(ptr), (n_))
    if (p->algorithm == QE_ALG_QEQEA) {
        ALLOC(a.slot, I * S);
        ALLOC(a.qrec, I * Q);
        // populations small enough for the shared-slot search in LDS: the
        // fused kernel commits the elitism of the slots one circuit alone used
        if (P * L <= (size_t)DEDUP_MAX_ENTRIES && L <= 256 && S < ((size_t)1 << 31)) {
            ALLOC(a.dup, 2 * I * P * L);
            ALLOC(a.shared_list, 2 * I * P * L);
            ALLOC(a.shared_count, 2 * I);
        }
        ALLOC(a.su3_tab, (size_t)4 * SU3_TAB);
    } else {
        ALLOC(a.genomes[0], (size_t)genes);
        ALLOC(a.genomes[1], (size_t)genes);
    }
    float* t32 = nullptr;
    double* t64 = nullptr;
    ALLOC(t32, (size_t)target_elems * 2);
    ALLOC(t64, (size_t)target_elems * 2);
    a.target32 = t32;
    a.target64 = t64;
    ALLOC(a.inst_best_f, I);
    if (p->algorithm == QE_ALG_QEQEA) {
        a.MW = (uint32_t)((P + 31) / 32);
        ALLOC(a.mutmask, 2 * I * a.MW);
    }
    ALLOC(a.inst_best_gates, I * L);
    ALLOC(a.inst_best_angles, I * L);
    ALLOC(c->gates, (size_t)genes);
    if (p->library == QE_LIB_ISING) ALLOC(c->angles, I * P * L);
    ALLOC(c->f, I * P);
    ALLOC(c->d_gen, 1);
    ALLOC(c->elite_cand, (int64_t)elite_cand_keys(I, P));
    ALLOC(c->check_word, 1);
    // mixed populations: per population and per circuit tables
    std::vector<int32_t> h_cgoff;
    std::vector<int64_t> h_goff, h_ctoff;
    std::vector<int8_t> h_cn;
    int32_t *d_in = nullptr, *d_iL = nullptr;
    int64_t *d_igoff = nullptr, *d_itoff = nullptr;
    if (mixed) {
        c->inst_n.assign(inst_n, inst_n + I);
        c->inst_L.assign(inst_L, inst_L + I);
        c->inst_toff.resize(I);
        h_goff.resize(I);
        h_cn.resize(I * P);
        h_cgoff.resize(I * P + 1);
        h_ctoff.resize(I * P);
        int64_t go = 0, to = 0;
        for (size_t i = 0; i < I; ++i) {
            h_goff[i] = go;
            c->inst_toff[i] = to;
            for (size_t k = 0; k < P; ++k) {
                h_cn[i * P + k] = (int8_t)inst_n[i];
                h_cgoff[i * P + k] = (int32_t)(go + (int64_t)k * inst_L[i]);
                h_ctoff[i * P + k] = to;
            }
            go += (int64_t)P * inst_L[i];
            to += (int64_t)1 << (2 * inst_n[i]);
        }
        h_cgoff[I * P] = (int32_t)go;
        ALLOC(d_in, I);
        ALLOC(d_iL, I);
        ALLOC(d_igoff, I);
        ALLOC(d_itoff, I);
        ALLOC(c->circ_n, I * P);
        ALLOC(c->circ_goff, I * P + 1);
        ALLOC(c->circ_toff, I * P);
        c->mix_work_bytes = qe_eval_workspace_bytes((int32_t)(I * P));
        ALLOC(c->mix_order, c->mix_work_bytes / sizeof(int32_t));
        ALLOC(c->mix_eval_work, c->mix_work_bytes / sizeof(int32_t));
        a.inst_n = d_in;
        a.inst_L = d_iL;
        a.inst_goff = d_igoff;
        a.inst_toff = d_itoff;
    }
#undef ALLOC
    if (st == QE_OK) st = device_error_word(&a.err);
    if (st != QE_OK) { std::string m = g_last_error; free_ctx(c); return fail(st, m); }
    a.gen_ptr = nullptr;
    hipError_t e = hipSuccess;
    if (mixed) {
        e = hipMemcpy(d_in, inst_n, I * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_iL, inst_L, I * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_igoff, h_goff.data(), I * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_itoff, c->inst_toff.data(), I * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->circ_n, h_cn.data(), I * P, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c->circ_goff, h_cgoff.data(), (I * P + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c->circ_toff, h_ctoff.data(), I * P * sizeof(int64_t), hipMemcpyHostToDevice);
        // the cost order of the circuits: widths and lengths never change
        c->mix_w5 = schedule_for(5, 32).waves;
        if (e == hipSuccess) e = launch_mix_sort(mixed_batch(c, c->gates), c->mix_order, nullptr);
    }
    if (p->algorithm == QE_ALG_QEQEA) {
        // SU(3) step tables: cos/sin of a*domain/4096, domain pi/2 (angles)
        // and 2 pi (phases), computed in double, rounded to float.
        std::vector<float> tab(4 * SU3_TAB);
        for (int k = 0; k < SU3_TAB; ++k) {
            const double th = (double)k * (3.14159265358979323846 / 2.0) / 4096.0;
            const double ph = (double)k * (2.0 * 3.14159265358979323846) / 4096.0;
            tab[k] = (float)std::cos(th);
            tab[SU3_TAB + k] = (float)std::sin(th);
            tab[2 * SU3_TAB + k] = (float)std::cos(ph);
            tab[3 * SU3_TAB + k] = (float)std::sin(ph);
        }
        if (e == hipSuccess)
            e = hipMemcpy((void*)a.su3_tab, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_qeqea_init(a, nullptr);
    } else if (e == hipSuccess) {
        e = launch_ga_init(a, nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(QE_ERR_DEVICE, std::string("context initialisation: ") + hipGetErrorString(e));
    }
    *out = c;
    return QE_OK;
}

}  // namespace

extern "C" {

qe_status qe_create(const qe_problem* p, qe_ctx** out) { return create_impl(p, nullptr, nullptr, out); }

qe_status qe_create_mixed(const qe_problem* p, const int32_t* n_qubits_host, const int32_t* lengths_host,
                          qe_ctx** out) {
    if (!n_qubits_host || !lengths_host) return fail(QE_ERR_INVALID, "NULL width or length table");
    return create_impl(p, n_qubits_host, lengths_host, out);
}

qe_status qe_destroy(qe_ctx* c) {
    if (!c) return fail(QE_ERR_INVALID, "ctx is NULL");
    const hipError_t e = hipDeviceSynchronize();   // work still queued may use the buffers
    free_ctx(c);
    if (e != hipSuccess) return fail(QE_ERR_DEVICE, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
    return QE_OK;
}

qe_status qe_set_targets(qe_ctx* c, const void* t, void* stream) {
    QE_TRY(check_ctx(c, false));
    if (!t) return fail(QE_ERR_INVALID, "targets is NULL");
    const size_t reals = (size_t)c->target_elems * 2;
    hipStream_t s = (hipStream_t)stream;
    if (c->prob.fitness_mode == QE_FIT_PHASE_INSENSITIVE) {
        // the mode needs targets whose entries have modulus 0 or 1: check them
        // in place, before they are taken
        BatchArgs b{};
        if (c->mixed) {
            b = mixed_batch(c, c->gates);
        } else {
            b.B = c->prob.n_instances;
            b.uniform_n = c->prob.n_qubits;
            b.uniform_L = 1;
            b.gates = c->gates;
            b.num_gates = b.B;
            b.tstride = (int64_t)c->N * c->N;
            b.num_telems = c->target_elems;
        }
        b.targets = t;
        b.mode = QE_FIT_PHASE_INSENSITIVE;
        b.err = c->check_word;
        uint32_t flags = 0;
        QE_HIP(hipMemsetAsync(c->check_word, 0, sizeof(uint32_t), s));
        QE_HIP(launch_target_check(b, true, c->f, nullptr, nullptr, s));
        QE_HIP(hipMemcpyAsync(&flags, c->check_word, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        QE_HIP(hipStreamSynchronize(s));
        if (flags & QE_DEVERR_TARGET)
            return fail(QE_ERR_UNSUPPORTED, "the phase-insensitive fitness needs targets whose entries have "
                                            "modulus 0 or 1 (permutations with phases)");
    }
    QE_HIP(hipMemcpyAsync((void*)c->la.target64, t, reals * sizeof(double), hipMemcpyDeviceToDevice, s));
    QE_HIP(launch_c128_to_c64(c->la.target64, (float*)c->la.target32, (int64_t)reals, s));
    c->targets_set = true;
    return QE_OK;
}

qe_status qe_sample(qe_ctx* c, uint64_t gen, uint32_t* slots, uint16_t* gates, uint32_t* angles,
                    void* stream) {
    QE_TRY(check_ctx(c, false));
    if (!gates) return fail(QE_ERR_INVALID, "gates is NULL");
    if (is_ising(c) && !angles) return fail(QE_ERR_INVALID, "the Ising library needs angles_dev");
    LoopArgs a = c->la;
    if (c->prob.algorithm == QE_ALG_QEQEA) {
        if (!slots) return fail(QE_ERR_INVALID, "slots is NULL");
        QE_HIP(launch_qeqea_sample(a, gen, slots, gates, is_ising(c) ? angles : nullptr,
                                   (hipStream_t)stream));
    } else {
        QE_HIP(launch_ga_copy(a, gen, gates, (hipStream_t)stream));
    }
    return QE_OK;
}

qe_status qe_eval_population(qe_ctx* c, const uint16_t* gates, const uint32_t* angles, float* f,
                             void* stream) {
    QE_TRY(check_ctx(c, true));
    if (!gates || !f) return fail(QE_ERR_INVALID, "NULL buffer");
    if (is_ising(c) && !angles) return fail(QE_ERR_INVALID, "the Ising library needs angles_dev");
    if (c->mixed)
        QE_HIP(launch_mix_eval(mixed_batch(c, gates), c->mix_order, f, nullptr, nullptr, (hipStream_t)stream));
    else
        QE_HIP(launch_eval_population(c->la, gates, is_ising(c) ? angles : nullptr, f, (hipStream_t)stream));
    return QE_OK;
}

qe_status qe_update(qe_ctx* c, uint64_t gen, const uint32_t* slots, const uint16_t* gates,
                    const uint32_t* angles, const float* f, void* stream) {
    QE_TRY(check_ctx(c, false));
    if (!f || !gates) return fail(QE_ERR_INVALID, "NULL buffer");
    if (is_ising(c) && !angles) return fail(QE_ERR_INVALID, "the Ising library needs angles_dev");
    hipStream_t s = (hipStream_t)stream;
    const bool fused = c->fused_gen >= 0 && (uint64_t)c->fused_gen == gen;
    c->fused_gen = -1;
    if (c->prob.algorithm == QE_ALG_QEQEA) {
        if (!slots && !fused)
            return fail(QE_ERR_STATE, "slots_dev NULL needs qe_sample_eval of the same generation just before");
        if (slots) QE_HIP(launch_scatter(c->la, gen, slots, f, s));
        if (!fused) {
            QE_TRY(prepare_decisions(c, gen, 1, s));
            QE_HIP(launch_mutation_decisions(c->la, gen, s));
        }
        // after qe_sample_eval with no slot array the fused kernel has committed
        // the unshared slots (the search's list names the shared ones), and
        // the update runs the next generation's search; with slots_dev every
        // entry's slot has its key (the elitism is the same, run again, for
        // the committed ones)
        const bool words = fused && !slots && c->la.dup != nullptr;
        QE_HIP(launch_qeqea_update(c->la, gen, slots, gates, is_ising(c) ? angles : nullptr, f, s, words,
                                   words));
        if (words) note_words(c, gen + 1);
    } else {
        QE_HIP(launch_ga_update(c->la, gen, f, s));
    }
    return QE_OK;
}

qe_status qe_generation(qe_ctx* c, uint64_t gen, float* f, void* stream) {
    QE_TRY(check_ctx(c, true));
    c->fused_gen = -1;
    QE_TRY(prepare_decisions(c, gen, 1, (hipStream_t)stream));
    if (c->prob.algorithm == QE_ALG_QEQEA) QE_TRY(ensure_words(c, gen, (hipStream_t)stream));
    QE_TRY(enqueue_generation(c, c->la, gen, f ? f : c->f, (hipStream_t)stream));
    note_words(c, gen + 1);
    return QE_OK;
}

qe_status qe_sample_eval(qe_ctx* c, uint64_t gen, uint32_t* slots, uint16_t* gates,
                         uint32_t* angles, float* f, void* stream) {
    QE_TRY(check_ctx(c, true));
    if (c->prob.algorithm != QE_ALG_QEQEA) return fail(QE_ERR_UNSUPPORTED, "qe_sample_eval is QEQEA only");
    if (!gates || !f) return fail(QE_ERR_INVALID, "NULL buffer");
    if (is_ising(c) && !angles) return fail(QE_ERR_INVALID, "the Ising library needs angles_dev");
    // the generation's mutation decisions are drawn here, as in qe_generation
    QE_TRY(prepare_decisions(c, gen, 1, (hipStream_t)stream));
    QE_TRY(ensure_words(c, gen, (hipStream_t)stream));
    QE_HIP(launch_qeqea_fused(c->la, gen, slots, gates, is_ising(c) ? angles : nullptr, f, true,
                              (hipStream_t)stream));
    c->fused_gen = (int64_t)gen;
    return QE_OK;
}

static qe_status graph_for(qe_ctx* c, int32_t n_gen, float* f_hist, hipGraphExec_t* out) {
    auto key = std::make_pair((int)n_gen, f_hist);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) { *out = it->second; return QE_OK; }
    LoopArgs a = c->la;
    a.gen_ptr = c->d_gen;
    const size_t IP = (size_t)c->prob.n_instances * c->prob.size_of_population;
    hipGraph_t g = nullptr;
    QE_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    qe_status st = QE_OK;
    // (each generation's update runs the next one's shared-slot search;
    // qe_run_graph provides the first generation's words)
    for (int j = 0; j < n_gen && st == QE_OK; ++j)
        st = enqueue_generation(c, a, (uint64_t)j, f_hist ? f_hist + j * IP : c->f, c->capture_stream);
    hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
    if (st != QE_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(QE_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(QE_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    // upload now, so that the first replay does not pay for it
    e = hipGraphUpload(ex, c->capture_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->capture_stream);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(ex);
        return fail(QE_ERR_DEVICE, std::string("graph upload: ") + hipGetErrorString(e));
    }
    c->graphs.emplace(key, ex);
    *out = ex;
    return QE_OK;
}

qe_status qe_graph_prepare(qe_ctx* c, int32_t n_gen, float* f_hist) {
    QE_TRY(check_ctx(c, true));
    if (n_gen < 1) return fail(QE_ERR_INVALID, "n_gen must be >= 1");
    hipGraphExec_t ex;
    return graph_for(c, n_gen, f_hist, &ex);
}

qe_status qe_run_graph(qe_ctx* c, uint64_t first_gen, int32_t n_gen, float* f_hist, void* stream) {
    QE_TRY(check_ctx(c, true));
    if (n_gen < 1) return fail(QE_ERR_INVALID, "n_gen must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    hipGraphExec_t ex;
    QE_TRY(graph_for(c, n_gen, f_hist, &ex));
    c->fused_gen = -1;
    QE_TRY(prepare_decisions(c, first_gen, (uint64_t)n_gen, s));
    if (c->prob.algorithm == QE_ALG_QEQEA) QE_TRY(ensure_words(c, first_gen, s));
    QE_HIP(launch_gen_set(c->d_gen, first_gen, s));
    QE_HIP(hipGraphLaunch(ex, s));
    note_words(c, first_gen + (uint64_t)n_gen - 1);
    note_words(c, first_gen + (uint64_t)n_gen);
    return QE_OK;
}

qe_status qe_elite_recheck(qe_ctx* c, const uint16_t* gates, const uint32_t* angles, const float* f,
                           int32_t k, int32_t* idx, double* f64, void* stream) {
    QE_TRY(check_ctx(c, true));
    if (!f || !idx || !f64) return fail(QE_ERR_INVALID, "NULL buffer");
    if (!gates) {
        gates = c->gates;
        angles = c->angles;
    } else if (is_ising(c) && !angles) {
        return fail(QE_ERR_INVALID, "the Ising library needs angles_dev");
    }
    if (!is_ising(c)) angles = nullptr;
    if (k < 1 || k > c->prob.size_of_population) return fail(QE_ERR_INVALID, "k must be 1..P");
    if (c->prob.size_of_population > 4096) return fail(QE_ERR_UNSUPPORTED, "elite selection needs P <= 4096");
    hipStream_t s = (hipStream_t)stream;
    QE_HIP(launch_elite_select(c->la, f, k, idx, c->elite_cand, s));
    QE_HIP(launch_elite_eval(c->la, gates, angles, k, idx, f64, s));
    return QE_OK;
}

qe_status qe_get_best(qe_ctx* c, int32_t inst, uint16_t* gates_host, uint32_t* angles_host,
                      float* f32_host, double* f64_host) {
    QE_TRY(check_ctx(c, false));
    if (inst < 0 || inst >= c->prob.n_instances) return fail(QE_ERR_INVALID, "instance out of range");
    QE_HIP(hipDeviceSynchronize());
    // rows of the best-circuit table hold size_of_individual entries (the
    // longest genome of mixed populations); population inst uses its own L
    const int row = c->prob.size_of_individual;
    const int L = c->mixed ? c->inst_L[inst] : row;
    const int n = c->mixed ? c->inst_n[inst] : c->prob.n_qubits;
    const int64_t toff = c->mixed ? c->inst_toff[inst] : (int64_t)inst * c->N * c->N;
    float fv = 0;
    QE_HIP(hipMemcpy(&fv, c->la.inst_best_f + inst, sizeof(float), hipMemcpyDeviceToHost));
    if (gates_host)
        QE_HIP(hipMemcpy(gates_host, c->la.inst_best_gates + (size_t)inst * row, L * sizeof(uint16_t),
                         hipMemcpyDeviceToHost));
    if (angles_host)
        QE_HIP(hipMemcpy(angles_host, c->la.inst_best_angles + (size_t)inst * row, L * sizeof(uint32_t),
                         hipMemcpyDeviceToHost));
    if (f32_host) *f32_host = fv;
    if (f64_host) {
        if (!c->targets_set) return fail(QE_ERR_STATE, "qe_set_targets has not been called");
        qe_batch b{};
        b.num_circuits = 1;
        b.uniform_n = n;
        b.uniform_L = L;
        b.gates_dev = c->la.inst_best_gates + (size_t)inst * row;
        b.num_gates = L;
        b.target_stride = 0;
        b.targets_dev = c->la.target64 + (size_t)2 * toff;
        b.num_target_elems = (int64_t)1 << (2 * n);
        b.fitness_mode = c->prob.fitness_mode;
        b.angles_dev = is_ising(c) ? c->la.inst_best_angles + (size_t)inst * row : nullptr;
        double* d = nullptr;
        QE_HIP(hipMalloc(&d, sizeof(double)));
        qe_status st = qe_eval_fitness_fp64(&b, d, nullptr, nullptr, nullptr);
        hipError_t e = st == QE_OK ? hipMemcpy(f64_host, d, sizeof(double), hipMemcpyDeviceToHost) : hipSuccess;
        (void)hipFree(d);
        if (st != QE_OK) return st;
        if (e != hipSuccess) return fail(QE_ERR_DEVICE, hipGetErrorString(e));
    }
    if (!(fv == fv)) return fail(QE_ERR_NUMERIC, "best fitness is NaN");
    return QE_OK;
}

}  // extern "C"

// ------------------------------------------------------ checkpoint / restore
namespace {
struct Section {
    void* ptr;
    size_t bytes;
};

std::vector<Section> state_sections(qe_ctx* c) {
    const LoopArgs& a = c->la;
    const size_t I = c->prob.n_instances, L = c->prob.size_of_individual;
    std::vector<Section> v;
    if (c->prob.algorithm == QE_ALG_QEQEA) {
        v.push_back({a.slot, I * c->S * sizeof(SlotRec)});
        v.push_back({a.qrec, I * c->Q * sizeof(QutritRec)});
    } else {
        v.push_back({a.genomes[0], (size_t)c->genes * 2});
        v.push_back({a.genomes[1], (size_t)c->genes * 2});
    }
    v.push_back({a.inst_best_f, I * 4});
    v.push_back({a.inst_best_gates, I * L * 2});
    v.push_back({a.inst_best_angles, I * L * 4});
    return v;
}

// Field by field (a caller's struct may carry arbitrary padding bytes, and
// +0 and -0 are the same parameter value).
bool same_problem(const qe_problem& x, const qe_problem& y) {
    return x.n_qubits == y.n_qubits && x.library == y.library && x.algorithm == y.algorithm &&
           x.size_of_individual == y.size_of_individual &&
           x.size_of_population == y.size_of_population && x.n_instances == y.n_instances &&
           x.prob_mutation == y.prob_mutation && x.mutation_range == y.mutation_range &&
           x.ga_crossover_prob == y.ga_crossover_prob &&
           x.ga_gene_mutation_prob == y.ga_gene_mutation_prob && x.seed == y.seed &&
           x.fitness_mode == y.fitness_mode;
}

// Identifies the per-population widths and lengths of a mixed context
// (FNV-1a over both tables, never 0); 0 for a uniform one.
uint32_t layout_tag(const qe_ctx* c) {
    if (!c->mixed) return 0u;
    uint32_t h = 2166136261u;
    auto mix = [&h](int32_t v) {
        for (int b = 0; b < 4; ++b) { h ^= (uint32_t)(v >> (8 * b)) & 0xFFu; h *= 16777619u; }
    };
    for (int32_t v : c->inst_n) mix(v);
    for (int32_t v : c->inst_L) mix(v);
    return h | 1u;
}

struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t layout;       // layout_tag of the context
    qe_problem prob;
    uint64_t payload;
};
}  // namespace

extern "C" {

qe_status qe_checkpoint(qe_ctx* c, void* buf, size_t* size) {
    QE_TRY(check_ctx(c, false));
    if (!size) return fail(QE_ERR_INVALID, "size is NULL");
    auto secs = state_sections(c);
    size_t payload = 0;
    for (auto& s : secs) payload += s.bytes;
    const size_t need = sizeof(CkptHeader) + payload;
    if (!buf) { *size = need; return QE_OK; }
    if (*size < need) return fail(QE_ERR_INVALID, "checkpoint buffer too small");
    QE_HIP(hipDeviceSynchronize());
    CkptHeader h{};
    std::memcpy(h.magic, "QECKPT04", 8);
    h.version = 4;
    h.prob = c->prob;
    h.layout = layout_tag(c);
    h.payload = payload;
    std::memcpy(buf, &h, sizeof(h));
    char* p = static_cast<char*>(buf) + sizeof(h);
    for (auto& s : secs) {
        QE_HIP(hipMemcpy(p, s.ptr, s.bytes, hipMemcpyDeviceToHost));
        p += s.bytes;
    }
    *size = need;
    return QE_OK;
}

qe_status qe_restore(qe_ctx* c, const void* buf, size_t size) {
    QE_TRY(check_ctx(c, false));
    if (!buf || size < sizeof(CkptHeader)) return fail(QE_ERR_INVALID, "checkpoint too small");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "QECKPT04", 8) != 0 || h.version != 4)
        return fail(QE_ERR_INVALID, "not a libqe checkpoint");
    if (!same_problem(h.prob, c->prob) || h.layout != layout_tag(c))
        return fail(QE_ERR_INVALID, "checkpoint was written for a different problem");
    c->fused_gen = -1;
    auto secs = state_sections(c);
    size_t payload = 0;
    for (auto& s : secs) payload += s.bytes;
    if (h.payload != payload || size < sizeof(h) + payload) return fail(QE_ERR_INVALID, "checkpoint size mismatch");
    QE_HIP(hipDeviceSynchronize());
    const char* p = static_cast<const char*>(buf) + sizeof(h);
    for (auto& s : secs) {
        QE_HIP(hipMemcpy(s.ptr, p, s.bytes, hipMemcpyHostToDevice));
        p += s.bytes;
    }
    QE_HIP(hipDeviceSynchronize());
    c->next_decision_gen = ~0ull;   // the decision masks start cleared again
    return QE_OK;
}

qe_status qe_state_read(qe_ctx* c, int32_t which, void* dst, int64_t* elems, void* stream) {
    QE_TRY(check_ctx(c, false));
    if (!elems) return fail(QE_ERR_INVALID, "elems is NULL");
    const LoopArgs& a = c->la;
    const size_t I = c->prob.n_instances;
    const bool q = c->prob.algorithm == QE_ALG_QEQEA;
    int64_t n = 0;
    switch (which) {
        case 0: case 2: case 3: n = q ? (int64_t)(I * c->S) : 0; break;
        case 1: case 4: n = q ? (int64_t)(I * c->Q * 6) : 0; break;
        case 5: case 6: n = q ? 0 : c->genes; break;
        case 7: n = q ? (int64_t)(2 * I * a.MW) : 0; break;
        default: return fail(QE_ERR_INVALID, "unknown state field");
    }
    *elems = n;
    if (!dst || n == 0) return QE_OK;
    hipStream_t s = (hipStream_t)stream;
    if (which == 7)
        QE_HIP(hipMemcpyAsync(dst, a.mutmask, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    else if (which >= 5)
        QE_HIP(hipMemcpyAsync(dst, a.genomes[which - 5], (size_t)n * sizeof(uint16_t),
                              hipMemcpyDeviceToDevice, s));
    else
        QE_HIP(launch_state_gather(a, which, dst, s));
    return QE_OK;
}

}  // extern "C"
