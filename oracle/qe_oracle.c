/*
 * qe_oracle.c -- plain CPU oracle for the circuit-fitness path of
 * Krylov & Lukac, "Quantum Encoded Quantum Evolutionary Algorithm for the
 * Design of Quantum Circuits" (arXiv:1809.11134).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * What is computed, and in which precision:
 *   - circuit unitaries and the fitness of Eq. 11 (Sec. IV-E) in IEEE double,
 *     by one left-multiplication per gate, the gate embedded on its wires with
 *     the big-endian register convention of Eqs. 1-2 (Sec. III), for the
 *     discrete libraries and for the Ising gate model (Eqs. 3-6);
 *   - the counter-based random numbers (Philox4x32-10, Salmon et al., SC'11);
 *   - circuit construction by sampling (Sec. IV-D, Eq. 10), qutrit
 *     measurement (Sec. IV-A/IV-C step 1), segment fitness and elitism
 *     (Sec. IV-E.1), adaptive qubit mutation and SU(3) qutrit mutation
 *     (Sec. IV-F, Eq. 12), and the classical GA of Sec. V-B (SUS selection,
 *     two-point crossover, gene mutation).  The encoding state of these steps
 *     is single precision by the reading documented with the build, so these
 *     functions use IEEE float arithmetic written operation by operation and
 *     must be compiled with -ffp-contract=off.
 *
 * Parity status of each function is recorded next to it ("pinned by ..." or
 * "parity unpinned").
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QEO_API __attribute__((visibility("default")))

#define PI 3.14159265358979323846

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Pinned by the published known-answer vectors. */
/* ------------------------------------------------------------------------ */
QEO_API void qeo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {               /* Weyl key schedule */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream tags of the counter (word 0); word 1 = generation, word 2 =
 * population instance, word 3 = item. */
enum { TAG_SAMPLE = 1, TAG_MEASURE = 2, TAG_MUT_IND = 3, TAG_MUT_SLOT = 4,
       TAG_INIT = 5, TAG_GA_SUS = 6, TAG_GA_XOVER = 7, TAG_GA_MUT = 8 };

static void draw(uint64_t seed, uint32_t tag, uint32_t gen, uint32_t inst, uint32_t item,
                 uint32_t w[4])
{
    uint32_t c[4] = { tag, gen, inst, item };
    uint32_t k[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    qeo_philox4x32_10(c, k, w);
}

/* A uniform integer in [0, range) from one 32-bit word: floor(w * range / 2^32). */
static uint32_t scale_u32(uint32_t w, uint32_t range)
{
    return (uint32_t)(((uint64_t)w * range) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Gate library.  A gate is a 16-bit descriptor: kind in bits 0-3, target    */
/* wire in bits 4-7, control wire in bits 8-11.  Wire w is bit (n-1-w) of a  */
/* basis-state index: the first Kronecker factor is the most significant     */
/* one (Eq. 1), so X on the first qubit exchanges the two halves (Eq. 2).    */
/* ------------------------------------------------------------------------ */
enum { K_I = 0, K_NOT = 1, K_CNOT = 2, K_CV = 3, K_CVDG = 4, K_H = 5, K_T = 6,
       K_RX = 7, K_RY = 8, K_RZ = 9, K_ZZ = 10 };

static uint16_t mkdesc(int kind, int tgt, int ctl)
{
    return (uint16_t)(kind | (tgt << 4) | (ctl << 8));
}

/* 2x2 unitary acting on the target qubit (textbook definitions:
 * X; V = sqrt(X) = (1/2)[[1+i, 1-i], [1-i, 1+i]]; V^dagger; Hadamard;
 * T = diag(1, e^{i pi/4})). */
static void gate_matrix(int kind, cplx G[2][2])
{
    const double h = 0.5, r = 1.0 / sqrt(2.0);
    switch (kind) {
    case K_NOT: case K_CNOT:
        G[0][0] = 0; G[0][1] = 1; G[1][0] = 1; G[1][1] = 0; break;
    case K_CV:
        G[0][0] = h * (1 + I); G[0][1] = h * (1 - I);
        G[1][0] = h * (1 - I); G[1][1] = h * (1 + I); break;
    case K_CVDG:
        G[0][0] = h * (1 - I); G[0][1] = h * (1 + I);
        G[1][0] = h * (1 + I); G[1][1] = h * (1 - I); break;
    case K_H:
        G[0][0] = r; G[0][1] = r; G[1][0] = r; G[1][1] = -r; break;
    case K_T:
        G[0][0] = 1; G[0][1] = 0; G[1][0] = 0; G[1][1] = cexp(I * PI / 4); break;
    default:
        G[0][0] = 1; G[0][1] = 0; G[1][0] = 0; G[1][1] = 1; break;
    }
}

static int is_controlled(int kind) { return kind == K_CNOT || kind == K_CV || kind == K_CVDG; }

/* Returns 0 if the descriptor names a valid gate on n wires. */
QEO_API int qeo_check_desc(int n, uint16_t d)
{
    int kind = d & 15, t = (d >> 4) & 15, c = (d >> 8) & 15;
    if (d >> 12) return -1;
    if (kind > K_T) return -1;
    if (kind == K_I) return 0;
    if (t >= n) return -1;
    if (is_controlled(kind) && (c >= n || c == t)) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Ising gate model (Sec. III, Eqs. 3-6): R_x, R_y, R_z on the target wire    */
/* and the two-qubit interaction J on the wire pair (target, control field).  */
/* Every gate carries an angle, a u32 fraction of a full turn:               */
/* theta = 2 pi u / 2^32 (exact in double), so angles live in [0, 2 pi) and  */
/* wrap modulo 2 pi as the mutation of Sec. IV-F requires.                   */
/* ------------------------------------------------------------------------ */
static int is_ising(int kind) { return kind >= K_RX && kind <= K_ZZ; }

static double angle_of(uint32_t u) { return 2.0 * PI * ((double)u / 4294967296.0); }

/* Returns 0 if the descriptor names a valid gate of either model on n wires
 * (J needs two distinct wires). */
QEO_API int qeo_check_desc_ising(int n, uint16_t d)
{
    int kind = d & 15, t = (d >> 4) & 15, c = (d >> 8) & 15;
    if (!is_ising(kind)) return qeo_check_desc(n, d);
    if (d >> 12) return -1;
    if (t >= n) return -1;
    if (kind == K_ZZ && (c >= n || c == t)) return -1;
    return 0;
}

/* Eqs. 3-5: R_x(theta) = [[cos, -i sin], [-i sin, cos]],
 * R_y(theta) = [[cos, -sin], [sin, cos]], R_z(theta) = diag(e^{-i theta/2},
 * e^{i theta/2}), cos and sin of theta / 2. */
static void rotation_matrix(int kind, double th, cplx G[2][2])
{
    double c = cos(th / 2.0), s = sin(th / 2.0);
    if (kind == K_RX) {
        G[0][0] = c; G[0][1] = -I * s; G[1][0] = -I * s; G[1][1] = c;
    } else if (kind == K_RY) {
        G[0][0] = c; G[0][1] = -s; G[1][0] = s; G[1][1] = c;
    } else {
        G[0][0] = cexp(-I * th / 2.0); G[0][1] = 0; G[1][0] = 0; G[1][1] = cexp(I * th / 2.0);
    }
}

/* M <- G M for an Ising gate d with angle u.  The rotations transform row
 * pairs like any single-qubit gate.  J on wires (a, b) is diagonal: by
 * Eq. 6, read with the exponent i theta (the printed e^{theta} lacks the i
 * that unitarity needs), J = e^{-i theta/2} diag(1, e^{i theta}, e^{i theta},
 * 1) on the two wires, so row i is multiplied by e^{-i theta/2} when the two
 * wire bits of i agree and by e^{-i theta/2} e^{i theta} when they differ. */
static void apply_ising(int n, uint16_t d, uint32_t u, cplx* M)
{
    int kind = d & 15;
    int N = 1 << n;
    int t = (d >> 4) & 15, c = (d >> 8) & 15;
    double th = angle_of(u);
    if (kind == K_ZZ) {
        cplx same = cexp(-I * th / 2.0), diff = cexp(-I * th / 2.0) * cexp(I * th);
        for (int i = 0; i < N; ++i) {
            int ba = (i >> (n - 1 - t)) & 1, bb = (i >> (n - 1 - c)) & 1;
            cplx z = ba == bb ? same : diff;
            for (int j = 0; j < N; ++j) M[(size_t)i * N + j] *= z;
        }
        return;
    }
    int tb = 1 << (n - 1 - t);
    cplx G[2][2];
    rotation_matrix(kind, th, G);
    for (int i0 = 0; i0 < N; ++i0) {
        if (i0 & tb) continue;
        int i1 = i0 | tb;
        for (int j = 0; j < N; ++j) {
            cplx a = M[(size_t)i0 * N + j], b = M[(size_t)i1 * N + j];
            M[(size_t)i0 * N + j] = G[0][0] * a + G[0][1] * b;
            M[(size_t)i1 * N + j] = G[1][0] * a + G[1][1] * b;
        }
    }
}

/* M <- G M for the gate d embedded on n wires; M is N x N, row-major.
 * Row pairs (i0, i1 = i0 | target bit) are transformed by the 2x2 matrix;
 * a controlled gate leaves rows whose control bit is 0 unchanged. */
static void apply_gate(int n, uint16_t d, cplx* M)
{
    int kind = d & 15;
    if (kind == K_I) return;
    int N = 1 << n;
    int t = (d >> 4) & 15, c = (d >> 8) & 15;
    int tb = 1 << (n - 1 - t);
    int cb = is_controlled(kind) ? 1 << (n - 1 - c) : 0;
    cplx G[2][2];
    gate_matrix(kind, G);
    for (int i0 = 0; i0 < N; ++i0) {
        if (i0 & tb) continue;
        if (cb && !(i0 & cb)) continue;
        int i1 = i0 | tb;
        for (int j = 0; j < N; ++j) {
            cplx a = M[(size_t)i0 * N + j], b = M[(size_t)i1 * N + j];
            M[(size_t)i0 * N + j] = G[0][0] * a + G[0][1] * b;
            M[(size_t)i1 * N + j] = G[1][0] * a + G[1][1] * b;
        }
    }
}

/* U = G_{L-1} ... G_1 G_0: the gate listed first acts first.  angles[l]
 * is the angle of gate l (u32 turn fraction; read for Ising kinds only);
 * with angles NULL only the discrete kinds are valid.
 * Output U (N*N complex doubles, row-major). Returns 0, or -1 on a bad gate. */
QEO_API int qeo_unitary_ang(int n, int L, const uint16_t* gates, const uint32_t* angles,
                            double* U_out)
{
    int N = 1 << n;
    cplx* U = (cplx*)U_out;
    for (int i = 0; i < N * N; ++i) U[i] = 0;
    for (int i = 0; i < N; ++i) U[(size_t)i * N + i] = 1;
    for (int l = 0; l < L; ++l) {
        if (angles ? qeo_check_desc_ising(n, gates[l]) : qeo_check_desc(n, gates[l])) return -1;
        if (is_ising(gates[l] & 15)) apply_ising(n, gates[l], angles[l], U);
        else apply_gate(n, gates[l], U);
    }
    return 0;
}

QEO_API int qeo_unitary(int n, int L, const uint16_t* gates, double* U_out)
{
    return qeo_unitary_ang(n, L, gates, NULL, U_out);
}

/* Eq. 11 of Sec. IV-E: fitness(S) = 1 - sqrt((size - |tr(S^dagger T)|) / size),
 * size = 2^n, |.| the complex modulus.
 *   g      = |tr(S^dagger T)| / size
 *   f_tr   = Eq. 11 evaluated literally (the radicand clamped at 0)
 *   delta  = (1/2) min_phi ||S - e^{i phi} T||_F^2, the minimiser being
 *            phi = arg tr(T^dagger S); for unitary S and T this equals
 *            size - |tr(S^dagger T)| exactly, so
 *   f      = 1 - sqrt(clamp(delta / size, 0, 1)) is Eq. 11 again.
 * Pinned by closed forms, the gate identities and brute force (tests). */
static void fitness_of(int n, const cplx* S, const cplx* T, double out[4])
{
    int N = 1 << n;
    size_t NN = (size_t)N * N;
    cplx tr = 0;
    for (size_t k = 0; k < NN; ++k) tr += conj(T[k]) * S[k];   /* tr(T^dagger S) */
    double a = cabs(tr);
    double g = a / N;
    double rad = (N - a) / N;
    double f_tr = 1.0 - sqrt(rad > 0 ? rad : 0);
    cplx ph = (a > 0) ? tr / a : 1.0;
    double delta = 0;
    for (size_t k = 0; k < NN; ++k) {
        cplx e = S[k] - ph * T[k];
        delta += creal(e) * creal(e) + cimag(e) * cimag(e);
    }
    delta *= 0.5;
    double q = delta / N;
    if (q < 0) q = 0;
    if (q > 1) q = 1;
    out[0] = 1.0 - sqrt(q);
    out[1] = g;
    out[2] = delta;
    out[3] = f_tr;
}

/* Fitness of one circuit against target T (N*N complex doubles); angles as
 * in qeo_unitary_ang.  out = {f, g, delta, f_trace}.  Returns 0 or -1 on a
 * bad gate. */
QEO_API int qeo_fitness_ang(int n, int L, const uint16_t* gates, const uint32_t* angles,
                            const double* T, double out[4])
{
    int N = 1 << n;
    cplx* S = (cplx*)malloc(sizeof(cplx) * N * N);
    if (!S) return -2;
    int rc = qeo_unitary_ang(n, L, gates, angles, (double*)S);
    if (rc == 0) fitness_of(n, S, (const cplx*)T, out);
    free(S);
    return rc;
}

QEO_API int qeo_fitness(int n, int L, const uint16_t* gates, const double* T, double out[4])
{
    return qeo_fitness_ang(n, L, gates, NULL, T, out);
}

/* Phase-insensitive fitness, the reading under which the paper's Table II
 * figure (and its Table III accuracy) reproduces; Eq. 11 as printed stays the
 * primary fitness:
 *   gP  = sum_ij |S_ij|^2 |T_ij|^2 / size
 *   rad = sum_ij |S_ij|^2 (1 - |T_ij|^2) / size  (= 1 - gP for unitary S,
 *         whose rows have unit norm; free of cancellation near gP = 1)
 *   fP  = 1 - sqrt(clamp(rad, 0, 1)).
 * out = {fP, gP, rad}.  Pinned by a closed form, phase invariance,
 * rad + gP = 1 and, for permutation targets, the off-diagonal energy of
 * S T^dagger (tests). */
static void fitness_pi_of(int n, const cplx* S, const cplx* T, double out[3])
{
    int N = 1 << n;
    size_t NN = (size_t)N * N;
    double gp = 0, rad = 0;
    for (size_t k = 0; k < NN; ++k) {
        double s2 = creal(S[k]) * creal(S[k]) + cimag(S[k]) * cimag(S[k]);
        double t2 = creal(T[k]) * creal(T[k]) + cimag(T[k]) * cimag(T[k]);
        gp += s2 * t2;
        rad += s2 * (1.0 - t2);
    }
    gp /= N;
    rad /= N;
    double q = rad < 0 ? 0 : (rad > 1 ? 1 : rad);
    out[0] = 1.0 - sqrt(q);
    out[1] = gp;
    out[2] = rad;
}

/* Phase-insensitive fitness of one circuit against target T; angles as in
 * qeo_unitary_ang.  out = {fP, gP, rad}.  Returns 0 or -1 on a bad gate. */
QEO_API int qeo_fitness_pi_ang(int n, int L, const uint16_t* gates, const uint32_t* angles,
                               const double* T, double out[3])
{
    int N = 1 << n;
    cplx* S = (cplx*)malloc(sizeof(cplx) * N * N);
    if (!S) return -2;
    int rc = qeo_unitary_ang(n, L, gates, angles, (double*)S);
    if (rc == 0) fitness_pi_of(n, S, (const cplx*)T, out);
    free(S);
    return rc;
}

QEO_API int qeo_fitness_pi(int n, int L, const uint16_t* gates, const double* T, double out[3])
{
    return qeo_fitness_pi_ang(n, L, gates, NULL, T, out);
}

/* A batch of circuits of uneven width and length: circuit b has n[b] wires,
 * gates[goff[b] .. goff[b+1]) and its target at targets + toff[b] (complex
 * elements).  out is [B][4] as in qeo_fitness.  Circuits run in parallel
 * over the host's cores when built with OpenMP.  Returns the number of
 * circuits with a bad gate. */
QEO_API int qeo_eval_batch(int B, const int8_t* nq, const int32_t* goff, const uint16_t* gates,
                           const int64_t* toff, const double* targets, double* out)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < B; ++b) {
        int rc = qeo_fitness(nq[b], goff[b + 1] - goff[b], gates + goff[b],
                             targets + 2 * toff[b], out + 4 * (size_t)b);
        if (rc) bad++;
    }
    return bad;
}

/* The same over circuits with angles (angles parallel to gates, NULL for
 * discrete circuits) and either fitness: mode 0 Eq. 11, out [B][4] =
 * {f, g, delta, f_trace}; mode 1 the phase-insensitive fitness, out [B][4] =
 * {fP, gP, rad, 0}.  Returns the number of circuits with a bad gate. */
QEO_API int qeo_eval_batch_ang(int B, const int8_t* nq, const int32_t* goff, const uint16_t* gates,
                               const uint32_t* angles, const int64_t* toff, const double* targets,
                               int mode, double* out)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < B; ++b) {
        const uint32_t* ab = angles ? angles + goff[b] : NULL;
        double* o = out + 4 * (size_t)b;
        int rc;
        if (mode == 1) {
            o[3] = 0.0;
            rc = qeo_fitness_pi_ang(nq[b], goff[b + 1] - goff[b], gates + goff[b], ab,
                                    targets + 2 * toff[b], o);
        } else {
            rc = qeo_fitness_ang(nq[b], goff[b + 1] - goff[b], gates + goff[b], ab,
                                 targets + 2 * toff[b], o);
        }
        if (rc) bad++;
    }
    return bad;
}

/* Threads the batch evaluator uses (OpenMP), for reporting. */
QEO_API int qeo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the batch evaluator (timing on one core). */
QEO_API void qeo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Gate-library instances (the enumeration order is a convention of this library): */
/*   library 0 {I, NOT, CNOT, CV, CV+}: I; NOT on wires 0..n-1; then for     */
/*     every ordered pair (c, t), c != t, lexicographic: CNOT, CV, CV+.      */
/*   library 1 {H, T, CNOT, CV, CV+}: H on wires 0..n-1; T on 0..n-1; then   */
/*     the same controlled triples.                                          */
/* ------------------------------------------------------------------------ */
QEO_API int qeo_lib_size(int lib, int n)
{
    int pairs = n * (n - 1);
    return lib == 0 ? 1 + n + 3 * pairs : 2 * n + 3 * pairs;
}

static void pair_of(int n, int p, int* c, int* t)
{
    *c = p / (n - 1);
    int tt = p % (n - 1);
    *t = tt < *c ? tt : tt + 1;
}

QEO_API uint16_t qeo_lib_desc(int lib, int n, int idx)
{
    int head = lib == 0 ? 1 + n : 2 * n;
    if (idx < head) {
        if (lib == 0) return idx == 0 ? mkdesc(K_I, 0, 0) : mkdesc(K_NOT, idx - 1, 0);
        return idx < n ? mkdesc(K_H, idx, 0) : mkdesc(K_T, idx - n, 0);
    }
    int p = (idx - head) / 3, which = (idx - head) % 3, c, t;
    pair_of(n, p, &c, &t);
    static const int kinds[3] = { K_CNOT, K_CV, K_CVDG };
    return mkdesc(kinds[which], t, c);
}

/* ------------------------------------------------------------------------ */
/* QEQEA encoding (Sec. IV-B, Fig. 4): per population instance, R = n + K    */
/* regions of L*P qubits, rotation regions r < n first; qutrits only for     */
/* rotation slots.  K counts the interaction templates: the C(n,2) unordered */
/* wire pairs for the Ising library (library 2), the n(n-1) ordered pairs    */
/* for the directed gates of libraries 0 and 1.                              */
/* Slot index s = r*L*P + ind*L + pos (Eq. 10).                              */
/* Qubit angle: u32 fraction of a full turn.  Qutrit: 3 complex amplitudes   */
/* stored as 6 floats (re0, im0, re1, im1, re2, im2).                        */
/* ------------------------------------------------------------------------ */
enum { LIB_ISING = 2 };

QEO_API int qeo_regions(int n, int lib)
{
    return lib == LIB_ISING ? n + n * (n - 1) / 2 : n * n;
}

/* Unordered wire pair k (a < b), lexicographic: (0,1), (0,2), ..., (1,2), ... */
static void upair_of(int n, int k, int* a, int* b)
{
    int x = 0;
    while (k >= n - 1 - x) { k -= n - 1 - x; ++x; }
    *a = x;
    *b = x + 1 + k;
}

QEO_API uint32_t qeo_segment_index(int L, int P, int region, int ind, int pos)
{
    return (uint32_t)region * (uint32_t)L * (uint32_t)P + (uint32_t)ind * (uint32_t)L + (uint32_t)pos;
}

/* Born-rule measurement of a qutrit with uniform u in [0,1) taken from the
 * top 24 bits of w; returns the axis index 0 (x), 1 (y) or 2 (z).  The
 * cumulative weights need no normalisation: u is scaled by their total.
 * Parity with the GPU is bit-exact by construction; the Born frequencies are
 * pinned by a test over the whole u grid. */
QEO_API int qeo_measure(const float* q, uint32_t w)
{
    float p0 = q[0] * q[0] + q[1] * q[1];
    float p1 = q[2] * q[2] + q[3] * q[3];
    float p2 = q[4] * q[4] + q[5] * q[5];
    float c0 = p0;
    float c1 = c0 + p1;
    float c2 = c1 + p2;
    float u = (float)(w >> 8) * 0x1p-24f;
    float x = u * c2;
    if (x < c0) return 0;
    if (x < c1) return 1;
    return 2;
}

/* Quarter-turn index of a u32 angle, rounded to the nearest quarter. */
static int quarter(uint32_t theta) { return (int)(((theta + 0x20000000u) >> 30) & 3u); }

/* Decode slot s of instance inst into a gate.
 * Ising library (Secs. IV-A, IV-C): a rotation slot on wire w becomes the
 * rotation about the measured axis (x, y, z for outcomes 0, 1, 2) on w, a
 * template slot on the unordered pair (a, b) the interaction J on (a, b);
 * either takes the slot's angle (*angle).
 * Discrete libraries (the reading for {I, NOT, CNOT, CV, CV+}): a rotation
 * slot on wire w becomes NOT_w when the measured axis is x and the angle is
 * a half turn (R_x(pi) = -iX), else the identity; a template slot on pair
 * (c, t) becomes the controlled V^q, q the angle in quarter turns: I, CV,
 * CNOT, CV+ (*angle = 0). */
QEO_API uint16_t qeo_decode_slot(int n, int lib, int L, int P, uint64_t seed, uint32_t gen,
                                 uint32_t inst, uint32_t s, const uint32_t* theta,
                                 const float* qutrit, uint32_t* angle)
{
    uint32_t LP = (uint32_t)L * (uint32_t)P;
    uint32_t r = s / LP;
    int q = quarter(theta[s]);
    *angle = 0;
    if (r < (uint32_t)n) {
        uint32_t w[4];
        draw(seed, TAG_MEASURE, gen, inst, s, w);
        int axis = qeo_measure(qutrit + 6 * (size_t)s, w[0]);
        if (lib == LIB_ISING) {
            *angle = theta[s];
            return mkdesc(K_RX + axis, (int)r, 0);
        }
        return (axis == 0 && q == 2) ? mkdesc(K_NOT, (int)r, 0) : mkdesc(K_I, 0, 0);
    }
    if (lib == LIB_ISING) {
        int a, b;
        upair_of(n, (int)(r - n), &a, &b);
        *angle = theta[s];
        return mkdesc(K_ZZ, a, b);
    }
    int c, t;
    pair_of(n, (int)(r - n), &c, &t);
    static const int kinds[4] = { K_I, K_CV, K_CNOT, K_CVDG };
    return q == 0 ? mkdesc(K_I, 0, 0) : mkdesc(kinds[q], t, c);
}

/* Circuit construction, Sec. IV-D: for each of the P circuits of each
 * instance and each position pos, draw whichIndividual in [0, P) and
 * whichRotationOrInteraction in [0, R), form the segment index of Eq. 10 and
 * decode that segment.  theta is [inst][S], qutrit [inst][n*L*P][6];
 * slots, gates and angles (may be NULL) are [inst][P][L].  Parity: bit-exact
 * (Eq. 10 pinned by the Table I example). */
QEO_API void qeo_qeqea_sample(int n, int lib, int L, int P, int I_, uint64_t seed, uint64_t gen64,
                              const uint32_t* theta, const float* qutrit,
                              uint32_t* slots, uint16_t* gates, uint32_t* angles)
{
    uint32_t gen = (uint32_t)gen64;
    uint32_t R = (uint32_t)qeo_regions(n, lib);
    size_t S = (size_t)R * L * P, Q = (size_t)n * L * P;
    for (int i = 0; i < I_; ++i) {
        for (int k = 0; k < P; ++k) {
            for (int pos = 0; pos < L; ++pos) {
                uint32_t w[4];
                draw(seed, TAG_SAMPLE, gen, (uint32_t)i, (uint32_t)(k * L + pos), w);
                uint32_t ind = scale_u32(w[0], (uint32_t)P);
                uint32_t region = scale_u32(w[1], R);
                uint32_t s = qeo_segment_index(L, P, (int)region, (int)ind, pos);
                size_t o = ((size_t)i * P + k) * L + pos;
                slots[o] = s;
                uint32_t ang;
                gates[o] = qeo_decode_slot(n, lib, L, P, seed, gen, (uint32_t)i, s, theta + i * S,
                                           qutrit + 6 * i * Q, &ang);
                if (angles) angles[o] = ang;
            }
        }
    }
}

/* Initial encoding: angles from the INIT stream, qutrits in the uniform
 * superposition (1,1,1)/sqrt(3), no best recorded yet (-1). */
QEO_API void qeo_qeqea_init(int n, int lib, int L, int P, int I_, uint64_t seed, uint32_t* theta,
                            float* qutrit, float* best_f, uint32_t* best_theta,
                            float* best_qutrit)
{
    size_t S = (size_t)qeo_regions(n, lib) * L * P, Q = (size_t)n * L * P;
    float a = (float)(1.0 / sqrt(3.0));
    for (int i = 0; i < I_; ++i) {
        for (size_t s = 0; s < S; ++s) {
            uint32_t w[4];
            draw(seed, TAG_INIT, 0xFFFFFFFFu, (uint32_t)i, (uint32_t)s, w);
            theta[i * S + s] = w[0];
            best_theta[i * S + s] = w[0];
            best_f[i * S + s] = -1.0f;
        }
        for (size_t s = 0; s < Q; ++s)
            for (int c = 0; c < 6; ++c) {
                float v = (c & 1) ? 0.0f : a;
                qutrit[6 * (i * Q + s) + c] = v;
                best_qutrit[6 * (i * Q + s) + c] = v;
            }
    }
}

/* Eq. 12 of Sec. IV-F: the SU(3) template built from three angles and five
 * phases, in double.  p = {th1, th2, th3, ph1, ph2, ph3, ph4, ph5}; U is 3x3
 * complex row-major (18 doubles).  Pinned by unitarity and det = 1. */
QEO_API void qeo_su3(const double* p, double* U_out)
{
    cplx* U = (cplx*)U_out;
    double c1 = cos(p[0]), s1 = sin(p[0]), c2 = cos(p[1]), s2 = sin(p[1]);
    double c3 = cos(p[2]), s3 = sin(p[2]);
    double f1 = p[3], f2 = p[4], f3 = p[5], f4 = p[6], f5 = p[7];
#define E(x) cexp(I * (x))
    U[0] = E(f1) * c1 * c2;
    U[1] = E(f3) * s1;
    U[2] = E(f4) * c1 * s2;
    U[3] = E(-f4 - f5) * s2 * s3 - E(f1 + f2 - f3) * s1 * c2 * c3;
    U[4] = E(f2) * c1 * c3;
    U[5] = -E(-f1 - f5) * c2 * s3 - E(f2 - f3 + f4) * s1 * s2 * c3;
    U[6] = -E(-f2 - f4) * s2 * c3 - E(f1 - f3 + f5) * s1 * c2 * s3;
    U[7] = E(f5) * c1 * s3;
    U[8] = E(-f1 - f2) * c2 * c3 - E(-f3 + f4 + f5) * s1 * s2 * s3;
#undef E
}

/* cos/sin of a*domain/4096 for a in [0, 4096): domain pi/2 for the angles,
 * 2 pi for the phases; computed in double and rounded to float. */
static float su3_tab[2][2][4096];   /* [angle|phase][cos|sin][a] */
static int su3_tab_ready = 0;
static void su3_tables(void)
{
    if (su3_tab_ready) return;
    for (int a = 0; a < 4096; ++a) {
        double th = (double)a * (PI / 2.0) / 4096.0;
        double ph = (double)a * (2.0 * PI) / 4096.0;
        su3_tab[0][0][a] = (float)cos(th);
        su3_tab[0][1][a] = (float)sin(th);
        su3_tab[1][0][a] = (float)cos(ph);
        su3_tab[1][1][a] = (float)sin(ph);
    }
    su3_tab_ready = 1;
}

/* One SU(3) mutation step on qutrit q (6 floats): Eq. 12 with only
 * parameter j non-zero, its value a*domain/4096.  With one parameter set
 * the template reduces to a real rotation in the (0,1), (0,2) or (1,2)
 * plane (th1, th2, th3), to diag(e^{i ph}, 1, e^{-i ph}) (ph1), to
 * diag(1, e^{i ph}, e^{-i ph}) (ph2), and to the identity for ph3..ph5,
 * which only multiply sine terms.  Float arithmetic, one rounding per
 * operation.  Pinned against qeo_su3 in the tests. */
QEO_API void qeo_su3_step(float* q, int j, int a)
{
    su3_tables();
    float x0 = q[0], y0 = q[1], x1 = q[2], y1 = q[3], x2 = q[4], y2 = q[5];
    if (j <= 2) {
        float c = su3_tab[0][0][a], s = su3_tab[0][1][a];
        if (j == 0) {          /* [[c, s, 0], [-s, c, 0], [0, 0, 1]] */
            q[0] = c * x0 + s * x1; q[1] = c * y0 + s * y1;
            q[2] = c * x1 - s * x0; q[3] = c * y1 - s * y0;
        } else if (j == 1) {   /* [[c, 0, s], [0, 1, 0], [-s, 0, c]] */
            q[0] = c * x0 + s * x2; q[1] = c * y0 + s * y2;
            q[4] = c * x2 - s * x0; q[5] = c * y2 - s * y0;
        } else {               /* [[1, 0, 0], [0, c, -s], [0, s, c]] */
            q[2] = c * x1 - s * x2; q[3] = c * y1 - s * y2;
            q[4] = s * x1 + c * x2; q[5] = s * y1 + c * y2;
        }
    } else if (j <= 4) {
        float c = su3_tab[1][0][a], s = su3_tab[1][1][a];
        if (j == 3) {          /* q0 *= e^{i ph} */
            q[0] = c * x0 - s * y0; q[1] = s * x0 + c * y0;
        } else {               /* q1 *= e^{i ph} */
            q[2] = c * x1 - s * y1; q[3] = s * x1 + c * y1;
        }
        /* q2 *= e^{-i ph} */
        q[4] = c * x2 + s * y2; q[5] = c * y2 - s * x2;
    }
}

/* Mutation threshold and step of the host-side parameters:
 * thr = floor(pm * 2^32); step scale = fl32(range / (2 pi) * 2^32). */
static uint64_t prob_threshold(double p)
{
    if (!(p > 0)) return 0;
    if (p >= 1) return (uint64_t)1 << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

/* Segment fitness, elitism and mutation for one generation
 * (Secs. IV-E.1 and IV-F), in the paper's order:
 *   1. every slot used to build a circuit gets that circuit's fitness; a
 *      slot used by several circuits keeps the largest;
 *   2. a used slot whose fitness beats its recorded best stores its state
 *      as the new best; otherwise its state reverts to the recorded best;
 *   3. each individual (ind < P) mutates with probability pm, either all its
 *      qubits (angle += or -= (1 - segFit) * range, wrapping mod 2 pi) or
 *      all its qutrits (one SU(3) step each), equiprobably; segFit is the
 *      slot's best fitness (0 if never used).
 * slots [inst][P][L] from qeo_qeqea_sample, f [inst][P] circuit fitness.
 * State arrays are updated in place.  Parity: bit-exact vs the GPU; the
 * trajectory itself is "parity unpinned" by the paper (invariants only). */
QEO_API void qeo_qeqea_update(int n, int lib, int L, int P, int I_, uint64_t seed, uint64_t gen64,
                              float pm, float range, const uint32_t* slots, const float* f,
                              uint32_t* theta, float* qutrit, float* best_f,
                              uint32_t* best_theta, float* best_qutrit)
{
    uint32_t gen = (uint32_t)gen64;
    uint32_t R = (uint32_t)qeo_regions(n, lib);
    size_t S = (size_t)R * L * P, Q = (size_t)n * L * P;
    uint64_t thr = prob_threshold((double)pm);
    float r32 = (float)((double)range / (2.0 * PI) * 4294967296.0);
    float* segfit = (float*)malloc(sizeof(float) * S);
    for (int i = 0; i < I_; ++i) {
        uint32_t* th = theta + i * S;
        uint32_t* bth = best_theta + i * S;
        float* bf = best_f + i * S;
        float* qu = qutrit + 6 * i * Q;
        float* bqu = best_qutrit + 6 * i * Q;
        /* 1. segment fitness */
        for (size_t s = 0; s < S; ++s) segfit[s] = -1.0f;
        for (int k = 0; k < P; ++k) {
            float fk = f[(size_t)i * P + k];
            if (!(fk >= 0.0f)) continue;          /* NaN never counts */
            for (int pos = 0; pos < L; ++pos) {
                uint32_t s = slots[((size_t)i * P + k) * L + pos];
                if (fk > segfit[s]) segfit[s] = fk;
            }
        }
        /* 2. elitism */
        for (size_t s = 0; s < S; ++s) {
            if (segfit[s] < 0.0f) continue;
            int rot = s < Q;
            if (segfit[s] > bf[s]) {
                bf[s] = segfit[s];
                bth[s] = th[s];
                if (rot) memcpy(bqu + 6 * s, qu + 6 * s, 6 * sizeof(float));
            } else {
                th[s] = bth[s];
                if (rot) memcpy(qu + 6 * s, bqu + 6 * s, 6 * sizeof(float));
            }
        }
        /* 3. mutation */
        for (int ind = 0; ind < P; ++ind) {
            uint32_t w[4];
            draw(seed, TAG_MUT_IND, gen, (uint32_t)i, (uint32_t)ind, w);
            if (!((uint64_t)w[0] < thr)) continue;
            int qutrit_mode = (int)(w[1] & 1u);
            for (uint32_t r = 0; r < R; ++r) {
                if (qutrit_mode && r >= (uint32_t)n) break;
                for (int pos = 0; pos < L; ++pos) {
                    uint32_t s = qeo_segment_index(L, P, (int)r, ind, pos);
                    float seg = bf[s] < 0.0f ? 0.0f : bf[s];
                    float om = 1.0f - seg;
                    uint32_t ws[4];
                    draw(seed, TAG_MUT_SLOT, gen, (uint32_t)i, s, ws);
                    if (!qutrit_mode) {
                        uint32_t d = (uint32_t)floorf(om * r32);
                        th[s] = (ws[0] & 1u) ? th[s] - d : th[s] + d;
                    } else {
                        int j = (int)scale_u32(ws[1], 8);
                        float u = (float)(ws[2] >> 8) * 0x1p-24f;
                        float x = u * om;
                        int a = (int)floorf(x * 4096.0f);
                        qeo_su3_step(qu + 6 * (size_t)s, j, a);
                    }
                }
            }
        }
    }
    free(segfit);
}

/* ------------------------------------------------------------------------ */
/* Classical GA of Sec. V-B for a discrete library: genome = L gate          */
/* descriptors; SUS selection, two-point crossover, gene mutation, and the   */
/* best individual carried over unchanged.  Parity: bit-exact vs the GPU;    */
/* SUS counts and crossover gene multisets are pinned by invariants; the     */
/* trajectory is "parity unpinned" by the paper.                             */
/* ------------------------------------------------------------------------ */
/* Initial genomes of population `inst` (P x L, uniform library instances
 * from the INIT stream). */
QEO_API void qeo_ga_init_at(int n, int lib, int L, int P, int inst, uint64_t seed, uint16_t* genomes)
{
    uint32_t nl = (uint32_t)qeo_lib_size(lib, n);
    for (int k = 0; k < P; ++k)
        for (int pos = 0; pos < L; ++pos) {
            uint32_t w[4];
            draw(seed, TAG_INIT, 0xFFFFFFFFu, (uint32_t)inst, (uint32_t)(k * L + pos), w);
            genomes[(size_t)k * L + pos] = qeo_lib_desc(lib, n, (int)scale_u32(w[0], nl));
        }
}

QEO_API void qeo_ga_init(int n, int lib, int L, int P, int I_, uint64_t seed, uint16_t* genomes)
{
    for (int i = 0; i < I_; ++i) qeo_ga_init_at(n, lib, L, P, i, seed, genomes + (size_t)i * P * L);
}

/* SUS over integer weights w_k = floor(f_k * 2^24): P equally spaced
 * pointers (r + k W) / P, r uniform in [0, W); pointer k selects the first
 * individual whose cumulative weight exceeds it.  sel[P] out. */
QEO_API void qeo_ga_sus(int P, const float* f, uint32_t w0, int32_t* sel)
{
    uint64_t* pre = (uint64_t*)malloc(sizeof(uint64_t) * (P + 1));
    pre[0] = 0;
    for (int k = 0; k < P; ++k) {
        uint32_t wk = (f[k] >= 0.0f) ? (uint32_t)floorf(f[k] * 16777216.0f) : 0u;
        pre[k + 1] = pre[k] + wk;
    }
    int uniform = pre[P] == 0;
    if (uniform)
        for (int k = 0; k <= P; ++k) pre[k] = (uint64_t)k;
    uint64_t W = pre[P];
    uint64_t r = (uint64_t)w0 * (W >> 32) + (((uint64_t)w0 * (W & 0xFFFFFFFFu)) >> 32);
    int m = 0;
    for (int k = 0; k < P; ++k) {
        uint64_t ptr = (r + (uint64_t)k * W) / (uint64_t)P;
        while (pre[m + 1] <= ptr) ++m;
        sel[k] = m;
    }
    free(pre);
}

/* One generation of the GA on population `inst` (its P fitness values fi and
 * its P x L genomes gi, updated in place). */
QEO_API void qeo_ga_update_at(int n, int lib, int L, int P, int inst, uint64_t seed, uint64_t gen64,
                              float pc, float pg, const float* fi, uint16_t* gi)
{
    uint32_t gen = (uint32_t)gen64;
    uint32_t nl = (uint32_t)qeo_lib_size(lib, n);
    uint64_t thr_c = prob_threshold((double)pc), thr_g = prob_threshold((double)pg);
    int32_t* sel = (int32_t*)malloc(sizeof(int32_t) * P);
    uint16_t* child = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)P * L);
    uint32_t i = (uint32_t)inst;
    int best = 0;                           /* lowest index among the maxima */
    float bv = -1.0f;                       /* NaN never counts */
    for (int k = 0; k < P; ++k)
        if (fi[k] > bv) { bv = fi[k]; best = k; }
    uint32_t w[4];
    draw(seed, TAG_GA_SUS, gen, i, 0u, w);
    qeo_ga_sus(P, fi, w[0], sel);
    for (int k = 0; k < P; ++k)
        memcpy(child + (size_t)k * L, gi + (size_t)sel[k] * L, sizeof(uint16_t) * L);
    /* two-point crossover: pair j mates children j and j + P/2 */
    int half = P / 2;
    for (int j = 0; j < half; ++j) {
        draw(seed, TAG_GA_XOVER, gen, i, (uint32_t)j, w);
        if (!((uint64_t)w[0] < thr_c)) continue;
        int a = (int)scale_u32(w[1], (uint32_t)(L + 1));
        int b = (int)scale_u32(w[2], (uint32_t)(L + 1));
        int lo = a < b ? a : b, hi = a < b ? b : a;
        for (int pos = lo; pos < hi; ++pos) {
            uint16_t t = child[(size_t)j * L + pos];
            child[(size_t)j * L + pos] = child[(size_t)(j + half) * L + pos];
            child[(size_t)(j + half) * L + pos] = t;
        }
    }
    /* gene mutation: a gene is replaced by a uniformly drawn instance */
    for (int k = 0; k < P; ++k)
        for (int pos = 0; pos < L; ++pos) {
            draw(seed, TAG_GA_MUT, gen, i, (uint32_t)(k * L + pos), w);
            if ((uint64_t)w[0] < thr_g)
                child[(size_t)k * L + pos] = qeo_lib_desc(lib, n, (int)scale_u32(w[1], nl));
        }
    /* elitism: the best individual survives unchanged in position 0 */
    memcpy(child, gi + (size_t)best * L, sizeof(uint16_t) * L);
    memcpy(gi, child, sizeof(uint16_t) * (size_t)P * L);
    free(sel);
    free(child);
}

QEO_API void qeo_ga_update(int n, int lib, int L, int P, int I_, uint64_t seed, uint64_t gen64,
                           float pc, float pg, const float* f, uint16_t* genomes)
{
    for (int i = 0; i < I_; ++i)
        qeo_ga_update_at(n, lib, L, P, i, seed, gen64, pc, pg, f + (size_t)i * P,
                         genomes + (size_t)i * P * L);
}
