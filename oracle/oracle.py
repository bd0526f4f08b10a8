"""ctypes binding of the C oracle (test infrastructure only).

All arrays are numpy arrays; complex matrices are complex128, row-major.
Builds ``liboracle.so`` on first use if it is missing.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("QE_ORACLE_LIB", _build.LIB)   # e.g. the sanitizer build
        if path == _build.LIB and not os.path.exists(path):
            _build.build_oracle()
        L = ctypes.CDLL(path)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        c = ctypes
        L.qeo_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.qeo_check_desc.argtypes = [c.c_int, c.c_uint16]
        L.qeo_check_desc_ising.argtypes = [c.c_int, c.c_uint16]
        u32p_or_null = c.c_void_p
        L.qeo_unitary_ang.argtypes = [c.c_int, c.c_int, u16p, u32p_or_null, f64p]
        L.qeo_fitness_ang.argtypes = [c.c_int, c.c_int, u16p, u32p_or_null, f64p, f64p]
        L.qeo_fitness_pi_ang.argtypes = [c.c_int, c.c_int, u16p, u32p_or_null, f64p, f64p]
        L.qeo_eval_batch.argtypes = [c.c_int, i8p, i32p, u16p, i64p, f64p, f64p]
        L.qeo_eval_batch_ang.argtypes = [c.c_int, i8p, i32p, u16p, u32p_or_null, i64p, f64p,
                                         c.c_int, f64p]
        L.qeo_regions.argtypes = [c.c_int, c.c_int]
        L.qeo_decode_slot.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                      c.c_uint32, c.c_uint32, c.c_uint32, u32p, f32p,
                                      ctypes.POINTER(c.c_uint32)]
        L.qeo_decode_slot.restype = c.c_uint16
        L.qeo_num_threads.restype = c.c_int
        L.qeo_set_num_threads.argtypes = [c.c_int]
        L.qeo_lib_size.argtypes = [c.c_int, c.c_int]
        L.qeo_lib_desc.argtypes = [c.c_int, c.c_int, c.c_int]
        L.qeo_lib_desc.restype = c.c_uint16
        L.qeo_segment_index.argtypes = [c.c_int] * 5
        L.qeo_segment_index.restype = c.c_uint32
        L.qeo_measure.argtypes = [f32p, c.c_uint32]
        L.qeo_qeqea_sample.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                       c.c_uint64, u32p, f32p, u32p, u16p, u32p_or_null]
        L.qeo_qeqea_init.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                     u32p, f32p, f32p, u32p, f32p]
        L.qeo_su3.argtypes = [f64p, f64p]
        L.qeo_su3_step.argtypes = [f32p, c.c_int, c.c_int]
        L.qeo_qeqea_update.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                       c.c_uint64, c.c_float, c.c_float, u32p, f32p,
                                       u32p, f32p, f32p, u32p, f32p]
        L.qeo_ga_init.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                  u16p]
        L.qeo_ga_init_at.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                     u16p]
        L.qeo_ga_update_at.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                       c.c_uint64, c.c_float, c.c_float, f32p, u16p]
        L.qeo_ga_sus.argtypes = [c.c_int, f32p, c.c_uint32, i32p]
        L.qeo_ga_update.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                    c.c_uint64, c.c_float, c.c_float, f32p, u16p]
        _lib = L
    return _lib


# --------------------------------------------------------------------------- RNG
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().qeo_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


# ------------------------------------------------------------------ gates, Eq. 11
RX, RY, RZ, ZZ = 7, 8, 9, 10          # Ising kinds (Eqs. 3-6)
LIB_ISING = 2


def desc(kind, tgt=0, ctl=0):
    return np.uint16(kind | (tgt << 4) | (ctl << 8))


def turns(theta):
    """u32 turn fraction of an angle in radians (rounded, modulo 2 pi)."""
    return np.uint32(int(round(theta / (2 * np.pi) * 2.0 ** 32)) % (1 << 32))


def check_desc(n, d, ising=False):
    f = lib().qeo_check_desc_ising if ising else lib().qeo_check_desc
    return f(n, int(d)) == 0


def _angles(angles, L):
    """(keep-alive array, pointer) for an optional angle array."""
    if angles is None:
        return None, None
    a = np.ascontiguousarray(angles, np.uint32)
    if len(a) != L:
        raise ValueError("one angle per gate")
    return a, (a.ctypes.data if L else np.zeros(1, np.uint32).ctypes.data)


def unitary(n, gates, angles=None):
    g = np.ascontiguousarray(gates, np.uint16)
    a, ap = _angles(angles, len(g))
    U = np.zeros((1 << n) * (1 << n) * 2, np.float64)
    rc = lib().qeo_unitary_ang(n, len(g), g, ap, U)
    if rc:
        raise ValueError("bad gate descriptor")
    return U.view(np.complex128).reshape(1 << n, 1 << n)


def fitness(n, gates, T, angles=None):
    """Returns (f, g, delta, f_trace) for one circuit against target T."""
    g = np.ascontiguousarray(gates, np.uint16)
    a, ap = _angles(angles, len(g))
    T = np.ascontiguousarray(T, np.complex128)
    out = np.zeros(4, np.float64)
    rc = lib().qeo_fitness_ang(n, len(g), g, ap, T.view(np.float64).ravel(), out)
    if rc:
        raise ValueError("bad gate descriptor")
    return tuple(float(x) for x in out)


def fitness_pi(n, gates, T, angles=None):
    """Phase-insensitive fitness: returns (fP, gP, radicand) for one circuit
    against target T (gP = sum |U_ij|^2 |T_ij|^2 / 2^n)."""
    g = np.ascontiguousarray(gates, np.uint16)
    a, ap = _angles(angles, len(g))
    T = np.ascontiguousarray(T, np.complex128)
    out = np.zeros(3, np.float64)
    rc = lib().qeo_fitness_pi_ang(n, len(g), g, ap, T.view(np.float64).ravel(), out)
    if rc:
        raise ValueError("bad gate descriptor")
    return tuple(float(x) for x in out)


def eval_batch(nq, goff, gates, toff, targets):
    """Uneven batch: returns an array [B, 4] of (f, g, delta, f_trace)."""
    nq = np.ascontiguousarray(nq, np.int8)
    goff = np.ascontiguousarray(goff, np.int32)
    gates = np.ascontiguousarray(gates, np.uint16)
    toff = np.ascontiguousarray(toff, np.int64)
    targets = np.ascontiguousarray(targets, np.complex128)
    B = len(nq)
    out = np.zeros((B, 4), np.float64)
    if len(gates) == 0:
        gates = np.zeros(1, np.uint16)
    bad = lib().qeo_eval_batch(B, nq, goff, gates, toff, targets.view(np.float64).ravel(), out)
    if bad:
        raise ValueError(f"{bad} circuits with bad gate descriptors")
    return out


def eval_batch_ang(nq, goff, gates, angles, toff, targets, mode=0):
    """Uneven batch with optional angles (None: discrete gates only); mode 0
    Eq. 11 -> rows (f, g, delta, f_trace), mode 1 phase-insensitive -> rows
    (fP, gP, radicand, 0)."""
    nq = np.ascontiguousarray(nq, np.int8)
    goff = np.ascontiguousarray(goff, np.int32)
    gates = np.ascontiguousarray(gates, np.uint16)
    toff = np.ascontiguousarray(toff, np.int64)
    targets = np.ascontiguousarray(targets, np.complex128)
    a, ap = _angles(angles, len(gates))
    B = len(nq)
    out = np.zeros((B, 4), np.float64)
    if len(gates) == 0:
        gates = np.zeros(1, np.uint16)
    bad = lib().qeo_eval_batch_ang(B, nq, goff, gates, ap, toff,
                                   targets.view(np.float64).ravel(), mode, out)
    if bad:
        raise ValueError(f"{bad} circuits with bad gate descriptors")
    return out


def num_threads():
    return lib().qeo_num_threads()


def set_num_threads(n):
    lib().qeo_set_num_threads(int(n))


# --------------------------------------------------------------------- libraries
def lib_size(library, n):
    return lib().qeo_lib_size(library, n)


def lib_table(library, n):
    return np.array([lib().qeo_lib_desc(library, n, i) for i in range(lib_size(library, n))],
                    np.uint16)


# ------------------------------------------------------------------------ QEQEA
def segment_index(L, P, region, ind, pos):
    return int(lib().qeo_segment_index(L, P, region, ind, pos))


def measure(q, w):
    return lib().qeo_measure(np.ascontiguousarray(q, np.float32), int(w))


def regions(n, library=0):
    return lib().qeo_regions(n, library)


def decode_slot(n, library, L, P, seed, gen, inst, s, theta, qutrit):
    """(descriptor, angle) of slot s; theta and qutrit are one instance's."""
    ang = ctypes.c_uint32(0)
    d = lib().qeo_decode_slot(n, library, L, P, seed, gen, inst, s,
                              np.ascontiguousarray(theta, np.uint32),
                              np.ascontiguousarray(qutrit, np.float32), ctypes.byref(ang))
    return int(d), int(ang.value)


class QeqeaState:
    """Encoding of I independent QEQEA populations (n wires, L, P, library)."""

    def __init__(self, n, L, P, I, seed, library=0):
        self.n, self.L, self.P, self.I, self.seed = n, L, P, I, seed
        self.library = library
        S = regions(n, library) * L * P
        Q = n * L * P
        self.theta = np.zeros(I * S, np.uint32)
        self.qutrit = np.zeros(I * Q * 6, np.float32)
        self.best_f = np.zeros(I * S, np.float32)
        self.best_theta = np.zeros(I * S, np.uint32)
        self.best_qutrit = np.zeros(I * Q * 6, np.float32)
        lib().qeo_qeqea_init(n, library, L, P, I, seed, self.theta, self.qutrit, self.best_f,
                             self.best_theta, self.best_qutrit)

    def copy(self):
        o = object.__new__(QeqeaState)
        o.__dict__.update({k: (v.copy() if isinstance(v, np.ndarray) else v)
                           for k, v in self.__dict__.items()})
        return o

    def sample(self, gen, with_angles=False):
        """(slots, gates) of generation gen, each [I*P, L]; with_angles adds
        the gates' angles (zero for discrete gates)."""
        n, L, P, I = self.n, self.L, self.P, self.I
        slots = np.zeros(I * P * L, np.uint32)
        gates = np.zeros(I * P * L, np.uint16)
        angles = np.zeros(I * P * L, np.uint32)
        lib().qeo_qeqea_sample(n, self.library, L, P, I, self.seed, gen, self.theta, self.qutrit,
                               slots, gates, angles.ctypes.data)
        out = (slots.reshape(I * P, L), gates.reshape(I * P, L))
        return out + (angles.reshape(I * P, L),) if with_angles else out

    def update(self, gen, pm, mrange, slots, f):
        lib().qeo_qeqea_update(self.n, self.library, self.L, self.P, self.I, self.seed, gen, pm,
                               mrange,
                               np.ascontiguousarray(slots, np.uint32).ravel(),
                               np.ascontiguousarray(f, np.float32).ravel(),
                               self.theta, self.qutrit, self.best_f, self.best_theta,
                               self.best_qutrit)


def su3(params):
    U = np.zeros(18, np.float64)
    lib().qeo_su3(np.ascontiguousarray(params, np.float64), U)
    return U.view(np.complex128).reshape(3, 3)


def su3_step(q, j, a):
    q = np.array(q, np.float32).copy()
    lib().qeo_su3_step(q, j, a)
    return q


# --------------------------------------------------------------------------- GA
def ga_init(n, library, L, P, I, seed):
    g = np.zeros(I * P * L, np.uint16)
    lib().qeo_ga_init(n, library, L, P, I, seed, g)
    return g.reshape(I * P, L)


def ga_sus(f, w0):
    f = np.ascontiguousarray(f, np.float32)
    sel = np.zeros(len(f), np.int32)
    lib().qeo_ga_sus(len(f), f, int(w0), sel)
    return sel


def ga_update(n, library, L, P, I, seed, gen, pc, pg, f, genomes):
    g = np.ascontiguousarray(genomes, np.uint16).ravel().copy()
    lib().qeo_ga_update(n, library, L, P, I, seed, gen, pc, pg,
                        np.ascontiguousarray(f, np.float32).ravel(), g)
    return g.reshape(I * P, L)


def ga_init_at(n, library, L, P, inst, seed):
    """Initial genomes [P, L] of population `inst` (the populations of a
    search are independent, each with its own width and length)."""
    g = np.zeros(P * L, np.uint16)
    lib().qeo_ga_init_at(n, library, L, P, inst, seed, g)
    return g.reshape(P, L)


def ga_update_at(n, library, L, P, inst, seed, gen, pc, pg, f, genomes):
    """One GA generation of population `inst`: f [P], genomes [P, L]."""
    g = np.ascontiguousarray(genomes, np.uint16).ravel().copy()
    lib().qeo_ga_update_at(n, library, L, P, inst, seed, gen, pc, pg,
                           np.ascontiguousarray(f, np.float32).ravel(), g)
    return g.reshape(P, L)
