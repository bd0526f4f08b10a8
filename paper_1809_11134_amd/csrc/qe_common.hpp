// Constants and small helpers shared by the libqe host code and kernels.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define QE_HD __host__ __device__
#else
#define QE_HD
#endif

namespace qe {

// Gate kinds of a descriptor (bits 0-3): the discrete libraries, then the
// Ising model of Sec. III (Eqs. 3-6), whose gates carry an angle: R_x, R_y,
// R_z on the target wire and the interaction J on the wire pair (target,
// control field).
enum : int { KIND_I = 0, KIND_NOT = 1, KIND_CNOT = 2, KIND_CV = 3, KIND_CVDG = 4, KIND_H = 5,
             KIND_T = 6, KIND_RX = 7, KIND_RY = 8, KIND_RZ = 9, KIND_ZZ = 10 };

QE_HD inline bool kind_controlled(int k) { return k == KIND_CNOT || k == KIND_CV || k == KIND_CVDG; }
QE_HD inline bool kind_ising(int k) { return k >= KIND_RX && k <= KIND_ZZ; }
// Gates on two wires: the controlled kinds and the interaction.
QE_HD inline bool kind_two_wire(int k) { return kind_controlled(k) || k == KIND_ZZ; }
QE_HD inline uint16_t make_desc(int kind, int tgt, int ctl) {
    return (uint16_t)(kind | (tgt << 4) | (ctl << 8));
}

// Philox stream tags (counter word 0).  Word 1 = generation, word 2 =
// population instance, word 3 = item.
enum : uint32_t { TAG_SAMPLE = 1, TAG_MEASURE = 2, TAG_MUT_IND = 3, TAG_MUT_SLOT = 4,
                  TAG_INIT = 5, TAG_GA_SUS = 6, TAG_GA_XOVER = 7, TAG_GA_MUT = 8 };
constexpr uint32_t GEN_INIT = 0xFFFFFFFFu;

// Ordered wire pair p of n wires (lexicographic over (c, t), t != c).
QE_HD inline void pair_of(int n, int p, int* c, int* t) {
    *c = p / (n - 1);
    const int tt = p % (n - 1);
    *t = tt < *c ? tt : tt + 1;
}

// Gate-library instances: library 0 = I, NOT(w), then per ordered pair
// (CNOT, CV, CV+); library 1 = H(w), T(w), then the same triples.
QE_HD inline int lib_size(int lib, int n) {
    return (lib == 0 ? 1 + n : 2 * n) + 3 * n * (n - 1);
}
QE_HD inline uint16_t lib_desc(int lib, int n, int idx) {
    const int head = lib == 0 ? 1 + n : 2 * n;
    if (idx < head) {
        if (lib == 0) return idx == 0 ? make_desc(KIND_I, 0, 0) : make_desc(KIND_NOT, idx - 1, 0);
        return idx < n ? make_desc(KIND_H, idx, 0) : make_desc(KIND_T, idx - n, 0);
    }
    const int p = (idx - head) / 3, which = (idx - head) % 3;
    int c, t;
    pair_of(n, p, &c, &t);
    const int kind = which == 0 ? KIND_CNOT : (which == 1 ? KIND_CV : KIND_CVDG);
    return make_desc(kind, t, c);
}

// Ising library (Secs. IV-A to IV-C): a rotation slot per wire and an
// interaction template per unordered wire pair.
constexpr int LIB_ISING = 2;

// Encoding regions of Eq. 10: n rotation regions, then one per template
// (the C(n,2) unordered pairs of the Ising library, the n(n-1) ordered
// pairs of the directed library gates).
QE_HD inline int regions(int n, int lib) { return lib == LIB_ISING ? n + n * (n - 1) / 2 : n * n; }

// Unordered wire pair k (a < b), lexicographic: (0,1), (0,2), ..., (1,2), ...
QE_HD inline void upair_of(int n, int k, int* a, int* b) {
    int x = 0;
    while (k >= n - 1 - x) {
        k -= n - 1 - x;
        ++x;
    }
    *a = x;
    *b = x + 1 + k;
}

constexpr int MAX_QUBITS = 6;
constexpr int SU3_TAB = 4096;   // entries of the SU(3) step tables

}  // namespace qe
