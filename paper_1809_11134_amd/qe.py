"""Python binding of libqe (ctypes).  Argument marshalling only: every step of
the path runs in the library's HIP kernels; torch supplies device memory and
streams.  Importing works without a GPU; calling needs libqe.so and a GPU, and
raises if either is missing (there is no CPU fallback)."""
import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qe.h")

QE_OK, QE_ERR_INVALID, QE_ERR_UNSUPPORTED, QE_ERR_DEVICE, QE_ERR_OOM, QE_ERR_NUMERIC, QE_ERR_STATE = range(7)
LIB_NCV, LIB_HT_NCV, LIB_ISING = 0, 1, 2
KIND_RX, KIND_RY, KIND_RZ, KIND_ZZ = 7, 8, 9, 10     # Ising kinds; angles are u32 turn fractions
ALG_QEQEA, ALG_GA = 0, 1
FIT_EQ11, FIT_PHASE_INSENSITIVE = 0, 1
(PATH_FP32, PATH_FP32_REG, PATH_FP32_LDS, PATH_MFMA_BF16, PATH_MFMA_FP16, PATH_MFMA_BF16_RAW,
 PATH_MFMA_FP16_RAW, PATH_DENSE) = range(8)
DEVERR_DESC, DEVERR_WIDTH, DEVERR_RANGE, DEVERR_NUMERIC, DEVERR_TARGET = 1, 2, 4, 8, 16


class QeError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class Batch(ctypes.Structure):
    _fields_ = [("num_circuits", ctypes.c_int32), ("uniform_n", ctypes.c_int32),
                ("n_qubits_dev", ctypes.c_void_p), ("uniform_L", ctypes.c_int32),
                ("gate_offsets_dev", ctypes.c_void_p), ("gates_dev", ctypes.c_void_p),
                ("num_gates", ctypes.c_int64), ("target_stride", ctypes.c_int64),
                ("target_offsets_dev", ctypes.c_void_p), ("targets_dev", ctypes.c_void_p),
                ("num_target_elems", ctypes.c_int64), ("fitness_mode", ctypes.c_int32),
                ("angles_dev", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("library", ctypes.c_int32),
                ("algorithm", ctypes.c_int32), ("size_of_individual", ctypes.c_int32),
                ("size_of_population", ctypes.c_int32), ("n_instances", ctypes.c_int32),
                ("prob_mutation", ctypes.c_float), ("mutation_range", ctypes.c_float),
                ("ga_crossover_prob", ctypes.c_float), ("ga_gene_mutation_prob", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("fitness_mode", ctypes.c_int32)]


_lib = None


def header_functions():
    """Names of the functions declared in include/qe.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qe_[a-z0-9_]+)\s*\(", text)))


def load():
    """Loads libqe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("QE_LIB", LIB_PATH)     # e.g. the host-sanitizer build
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1809_11134_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "qe_eval_fitness": [vp, P(Batch), i32, vp, vp, vp, vp],
        "qe_eval_fitness_fp64": [P(Batch), vp, vp, vp, vp],
        "qe_build_unitary": [P(Batch), i32, vp, i64, vp],
        "qe_device_errors": [P(i32)],
        "qe_create": [P(Problem), P(vp)],
        "qe_destroy": [vp],
        "qe_set_targets": [vp, vp, vp],
        "qe_sample": [vp, u64, vp, vp, vp, vp],
        "qe_eval_population": [vp, vp, vp, vp, vp],
        "qe_update": [vp, u64, vp, vp, vp, vp, vp],
        "qe_generation": [vp, u64, vp, vp],
        "qe_run_graph": [vp, u64, i32, vp, vp],
        "qe_sample_eval": [vp, u64, vp, vp, vp, vp, vp],
        "qe_graph_prepare": [vp, i32, vp],
        "qe_elite_recheck": [vp, vp, vp, vp, i32, vp, vp, vp],
        "qe_get_best": [vp, i32, vp, vp, P(ctypes.c_float), P(ctypes.c_double)],
        "qe_checkpoint": [vp, vp, P(ctypes.c_size_t)],
        "qe_restore": [vp, vp, ctypes.c_size_t],
        "qe_state_read": [vp, i32, vp, P(i64), vp],
        "qe_lib_table": [i32, i32, vp],
        "qe_set_schedule": [i32, i32],
        "qe_get_schedule": [i32, P(i32)],
        "qe_probe_lds": [i32, i32, i32, vp, P(ctypes.c_double), vp],
        "qe_probe_records": [i32, vp, i64, i64, ctypes.c_uint32, vp, vp],
        "qe_create_mixed": [P(Problem), vp, vp, P(vp)],
        "qe_eval_fitness_ws": [P(Batch), i32, vp, vp, vp, vp, ctypes.c_size_t, vp],
        "qe_eval_fitness_noalloc": [P(Batch), i32, vp, vp, vp, vp],
        "qe_set_schedule_ex": [i32, i32, i32, i32, i32],
        "qe_get_schedule_ex": [i32, i32, P(i32), P(i32), P(i32)],
        "qe_set_schedule_lib": [i32, i32, i32, i32, i32, i32],
        "qe_set_mfma_min_block": [i32, i32, i32],
        "qe_get_mfma_min_block": [i32, i32, P(i32)],
        "qe_get_schedule_lib": [i32, i32, i32, P(i32), P(i32), P(i32)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = i32
    L.qe_lib_size.argtypes = [i32, i32]
    L.qe_lib_size.restype = i32
    L.qe_eval_workspace_bytes.argtypes = [i32]
    L.qe_eval_workspace_bytes.restype = ctypes.c_size_t
    L.qe_last_error.restype = ctypes.c_char_p
    L.qe_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _call(name, *args):
    st = getattr(load(), name)(*args)
    if st != QE_OK:
        raise QeError(name, st, load().qe_last_error().decode())
    return st


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, dtype):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype:
        t = t.to(dtype)
    return t.contiguous()


def _gates(t):
    t = _dev(t, t.dtype if t.dtype == torch.int16 else torch.int32)
    if t.dtype != torch.int16:
        t = t.to(torch.int16)
    return t.contiguous()


def _angles(t):
    """Device angles as int32 storage of the u32 turn fractions."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != torch.int32:
        t = t.to(torch.int64) & 0xFFFFFFFF
        t = torch.where(t >= 1 << 31, t - (1 << 32), t).to(torch.int32)
    return t.contiguous()


def make_batch(gates, targets, n=None, L=None, nq=None, goff=None, toff=None, target_stride=None,
               fitness_mode=0, angles=None):
    """Builds a qe_batch from device tensors.  gates: int16/int32 descriptors
    ([B, L] for uniform lengths, flat with goff for uneven); targets: complex
    tensor ([T, N, N] or flat); n: uniform width or None with nq (int8 [B]);
    target_stride: complex elements between targets (0 = shared) or None with
    toff (int64 [B]); angles: None, or one u32 turn fraction per gate (int32
    storage, same shape as gates) for circuits with Ising gates."""
    keep = []
    b = Batch()
    g = _gates(gates)
    keep.append(g)
    a = _angles(angles)
    if a is not None:
        if a.numel() != g.numel():
            raise ValueError("one angle per gate")
        keep.append(a)
        b.angles_dev = a.data_ptr() if a.numel() else None
    if L is not None and goff is None:
        B = g.numel() // L if L > 0 else 0
        b.uniform_L = L
    else:
        goff = _dev(goff, torch.int32)
        keep.append(goff)
        B = goff.numel() - 1
        b.uniform_L = 0
        b.gate_offsets_dev = goff.data_ptr()
    b.num_circuits = B
    if n is not None:
        b.uniform_n = n
    else:
        nq = _dev(nq, torch.int8)
        keep.append(nq)
        b.uniform_n = 0
        b.n_qubits_dev = nq.data_ptr()
    b.gates_dev = g.data_ptr() if g.numel() else None
    b.num_gates = g.numel()
    b.fitness_mode = fitness_mode
    if targets is not None:
        t = targets.contiguous()
        keep.append(t)
        b.targets_dev = t.data_ptr()
        b.num_target_elems = t.numel()
        if target_stride is not None:
            b.target_stride = target_stride
        else:
            toff = _dev(toff, torch.int64)
            keep.append(toff)
            b.target_stride = -1
            b.target_offsets_dev = toff.data_ptr()
    return b, keep, B


def eval_workspace(B, device):
    """A device workspace for qe_eval_fitness_ws of B circuits (torch memory)."""
    nbytes = load().qe_eval_workspace_bytes(B)
    return torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=device)


def eval_fitness(gates, targets, n=None, L=None, nq=None, goff=None, toff=None, target_stride=0,
                 path=PATH_FP32, want_g=False, want_delta=False, stream=None, fitness_mode=0,
                 angles=None, workspace=True, ctx=None):
    """Eq. 11 fitness (or, with fitness_mode=FIT_PHASE_INSENSITIVE, the
    phase-insensitive fitness) of a batch on the FP32 or MFMA paths.  targets
    complex64; angles as in make_batch.  A mixed-width batch takes the
    cost-sorted single launch with a workspace (workspace=True: allocated
    here; or a tensor from eval_workspace) and one launch per width with
    workspace=False (qe_eval_fitness, lent ctx's workspace when ctx is a
    mixed context).  Returns (f, g or None, delta or None) as float32
    tensors."""
    targets = targets.to(torch.complex64) if targets.dtype != torch.complex64 else targets
    b, keep, B = make_batch(gates, targets, n, L, nq, goff, toff, target_stride, fitness_mode, angles)
    dev = targets.device
    f = torch.empty(B, dtype=torch.float32, device=dev)
    g = torch.empty(B, dtype=torch.float32, device=dev) if want_g else None
    d = torch.empty(B, dtype=torch.float32, device=dev) if want_delta else None
    if workspace is not False and n is None:
        ws = eval_workspace(B, dev) if workspace is True else workspace
        _call("qe_eval_fitness_ws", ctypes.byref(b), path, _ptr(f), _ptr(g), _ptr(d), _ptr(ws),
              ws.numel() * 4, _stream(stream))
    else:
        h = ctx.handle if ctx is not None else None
        _call("qe_eval_fitness", h, ctypes.byref(b), path, _ptr(f), _ptr(g), _ptr(d), _stream(stream))
    return f, g, d


def eval_fitness_fp64(gates, targets, n=None, L=None, nq=None, goff=None, toff=None,
                      target_stride=0, want_g=False, want_delta=False, stream=None, fitness_mode=0,
                      angles=None):
    targets = targets.to(torch.complex128) if targets.dtype != torch.complex128 else targets
    b, keep, B = make_batch(gates, targets, n, L, nq, goff, toff, target_stride, fitness_mode, angles)
    dev = targets.device
    f = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty(B, dtype=torch.float64, device=dev) if want_g else None
    d = torch.empty(B, dtype=torch.float64, device=dev) if want_delta else None
    _call("qe_eval_fitness_fp64", ctypes.byref(b), _ptr(f), _ptr(g), _ptr(d), _stream(stream))
    return f, g, d


def build_unitary(gates, n, L, precision=1, stream=None, angles=None):
    """Unitaries of B circuits of n wires and L gates: [B, N, N] complex."""
    b, keep, B = make_batch(gates, None, n=n, L=L, angles=angles)
    N = 1 << n
    dtype = torch.complex128 if precision == 1 else torch.complex64
    out = torch.empty((B, N, N), dtype=dtype, device=gates.device)
    _call("qe_build_unitary", ctypes.byref(b), precision, _ptr(out), out.numel(), _stream(stream))
    return out


def device_errors():
    v = ctypes.c_int32(0)
    _call("qe_device_errors", ctypes.byref(v))
    return v.value


def lib_table(library, n):
    size = load().qe_lib_size(library, n)
    buf = (ctypes.c_uint16 * size)()
    _call("qe_lib_table", library, n, buf)
    return [int(x) for x in buf]


def set_schedule(n, lds):
    _call("qe_set_schedule", n, int(lds))


def get_schedule(n):
    v = ctypes.c_int32(0)
    _call("qe_get_schedule", n, ctypes.byref(v))
    return v.value


def set_schedule_ex(n, lclass, lds, waves, cpb):
    """Full schedule of width n, length class lclass (0: L < 32, 1: L >= 32)."""
    _call("qe_set_schedule_ex", n, lclass, int(lds), int(waves), int(cpb))


def get_schedule_ex(n, lclass):
    """(lds, waves, cpb) of width n, length class lclass."""
    v = [ctypes.c_int32(0) for _ in range(3)]
    _call("qe_get_schedule_ex", n, lclass, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


SCHED_DISCRETE, SCHED_SAMPLED, SCHED_ISING = 0, 1, 2


def set_schedule_lib(n, lclass, lib_class, lds, waves, cpb):
    """Schedule of width n, length class lclass, library class lib_class
    (SCHED_DISCRETE, SCHED_SAMPLED, SCHED_ISING)."""
    _call("qe_set_schedule_lib", n, lclass, lib_class, int(lds), int(waves), int(cpb))


def set_mfma_min_block(n, lclass, min_block):
    """MFMA paths: groups of fewer than min_block gates go gate by gate in FP32."""
    _call("qe_set_mfma_min_block", n, lclass, int(min_block))


def get_mfma_min_block(n, lclass):
    v = ctypes.c_int32(0)
    _call("qe_get_mfma_min_block", n, lclass, ctypes.byref(v))
    return v.value


def get_schedule_lib(n, lclass, lib_class):
    """(lds, waves, cpb) of width n, length class lclass, library class lib_class."""
    v = [ctypes.c_int32(0) for _ in range(3)]
    _call("qe_get_schedule_lib", n, lclass, lib_class, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


class Context:
    """A QEQEA or GA search: ctx-owned encoding on the current device.
    widths / lengths (lists of I entries, GA only): populations of their own
    width and genome length (qe_create_mixed); n and L are then ignored."""

    def __init__(self, n, library, algorithm, L, P, instances=1, prob_mutation=0.1,
                 mutation_range=0.7853981633974483, ga_crossover_prob=0.9,
                 ga_gene_mutation_prob=None, seed=0, fitness_mode=0, widths=None, lengths=None):
        self.mixed = widths is not None
        if self.mixed:
            instances = len(widths)
            if lengths is None or len(lengths) != instances:
                raise ValueError("one genome length per population")
            n, L = max(widths), max(lengths)
            self.widths, self.lengths = [int(x) for x in widths], [int(x) for x in lengths]
        if ga_gene_mutation_prob is None:
            ga_gene_mutation_prob = 1.0 / L
        self.problem = Problem(n, library, algorithm, L, P, instances, prob_mutation,
                               mutation_range, ga_crossover_prob, ga_gene_mutation_prob, seed,
                               fitness_mode)
        self.n, self.L, self.P, self.I = n, L, P, instances
        self.algorithm = algorithm
        self.ising = library == LIB_ISING
        h = ctypes.c_void_p(0)
        if self.mixed:
            wn = (ctypes.c_int32 * instances)(*self.widths)
            wl = (ctypes.c_int32 * instances)(*self.lengths)
            _call("qe_create_mixed", ctypes.byref(self.problem), wn, wl, ctypes.byref(h))
            self.genes = P * sum(self.lengths)
        else:
            _call("qe_create", ctypes.byref(self.problem), ctypes.byref(h))
            self.genes = instances * P * L
        self.handle = h
        self._keep = []

    def close(self):
        if self.handle:
            _call("qe_destroy", self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def circuits(self):
        return self.I * self.P

    def set_targets(self, targets, stream=None):
        t = targets.to(torch.complex128).contiguous()
        self._keep = [t]
        _call("qe_set_targets", self.handle, _ptr(t), _stream(stream))

    def _new_angles(self):
        if not self.ising:
            return None
        return torch.empty((self.circuits, self.L), dtype=torch.int32,
                           device=torch.device("cuda", torch.cuda.current_device()))

    def sample(self, gen, stream=None):
        """(slots, gates), and for the Ising library (slots, gates, angles).
        Mixed populations: gates is flat, population by population."""
        dev = torch.device("cuda", torch.cuda.current_device())
        slots = torch.empty((self.circuits, self.L), dtype=torch.int32, device=dev)
        shape = (self.genes,) if self.mixed else (self.circuits, self.L)
        gates = torch.empty(shape, dtype=torch.int16, device=dev)
        angles = self._new_angles()
        _call("qe_sample", self.handle, gen, _ptr(slots), _ptr(gates), _ptr(angles), _stream(stream))
        return (slots, gates, angles) if self.ising else (slots, gates)

    def eval_population(self, gates, angles=None, stream=None):
        f = torch.empty(self.circuits, dtype=torch.float32, device=gates.device)
        _call("qe_eval_population", self.handle, _ptr(_gates(gates)), _ptr(_angles(angles)), _ptr(f),
              _stream(stream))
        return f

    def update(self, gen, slots, gates, f, angles=None, stream=None):
        """slots None: right after sample_eval(gen), which left the segment
        keys and decisions (the slots are drawn again)."""
        _call("qe_update", self.handle, gen, _ptr(slots), _ptr(_gates(gates)), _ptr(_angles(angles)),
              _ptr(f.contiguous()), _stream(stream))

    def generation(self, gen, f=None, stream=None):
        if f is None:
            f = torch.empty(self.circuits, dtype=torch.float32,
                            device=torch.device("cuda", torch.cuda.current_device()))
        _call("qe_generation", self.handle, gen, _ptr(f), _stream(stream))
        return f

    def sample_eval(self, gen, slots=None, gates=None, f=None, stream=None, angles=None,
                    keep_slots=True):
        """(slots, gates, f), and for the Ising library (slots, gates, angles, f);
        keep_slots=False leaves the slot indices out (slots is None)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        if slots is None and keep_slots:
            slots = torch.empty((self.circuits, self.L), dtype=torch.int32, device=dev)
        if gates is None:
            gates = torch.empty((self.circuits, self.L), dtype=torch.int16, device=dev)
        if f is None:
            f = torch.empty(self.circuits, dtype=torch.float32, device=dev)
        if angles is None:
            angles = self._new_angles()
        _call("qe_sample_eval", self.handle, gen, _ptr(slots), _ptr(gates), _ptr(angles), _ptr(f),
              _stream(stream))
        return (slots, gates, angles, f) if self.ising else (slots, gates, f)

    def graph_prepare(self, n_gen, f_hist=None):
        _call("qe_graph_prepare", self.handle, n_gen, _ptr(f_hist))

    def run_graph(self, first_gen, n_gen, f_hist=None, stream=None):
        _call("qe_run_graph", self.handle, first_gen, n_gen, _ptr(f_hist), _stream(stream))

    def elite_recheck(self, gates, f, k, stream=None, angles=None):
        idx = torch.empty((self.I, k), dtype=torch.int32, device=f.device)
        f64 = torch.empty((self.I, k), dtype=torch.float64, device=f.device)
        _call("qe_elite_recheck", self.handle, _ptr(_gates(gates) if gates is not None else None),
              _ptr(_angles(angles)), _ptr(f.contiguous()), k,
              _ptr(idx), _ptr(f64), _stream(stream))
        return idx, f64

    def get_best(self, instance=0, with_fp64=True, with_angles=False):
        """(gates, f32, f64 or None), with_angles adding the gates' angles."""
        gates = (ctypes.c_uint16 * self.L)()
        angles = (ctypes.c_uint32 * self.L)()
        f32 = ctypes.c_float(0)
        f64 = ctypes.c_double(0)
        _call("qe_get_best", self.handle, instance, gates, angles, ctypes.byref(f32),
              ctypes.byref(f64) if with_fp64 else None)
        L = self.lengths[instance] if self.mixed else self.L
        out = ([int(x) for x in gates[:L]], f32.value, (f64.value if with_fp64 else None))
        return out + ([int(x) for x in angles[:L]],) if with_angles else out

    def checkpoint(self):
        size = ctypes.c_size_t(0)
        _call("qe_checkpoint", self.handle, None, ctypes.byref(size))
        buf = ctypes.create_string_buffer(size.value)
        _call("qe_checkpoint", self.handle, buf, ctypes.byref(size))
        return bytes(buf.raw[:size.value])

    def restore(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _call("qe_restore", self.handle, buf, len(blob))

    _VIEWS = {"theta": (0, torch.int32), "qutrit": (1, torch.float32), "best_f": (2, torch.float32),
              "best_theta": (3, torch.int32), "best_qutrit": (4, torch.float32),
              "genomes0": (5, torch.int16), "genomes1": (6, torch.int16),
              "mutation_masks": (7, torch.int32)}

    def state(self, name, stream=None):
        """A device copy of one field of the ctx-owned state."""
        which, dtype = self._VIEWS[name]
        n = ctypes.c_int64(0)
        _call("qe_state_read", self.handle, which, None, ctypes.byref(n), None)
        out = torch.empty(n.value, dtype=dtype, device=torch.device("cuda", torch.cuda.current_device()))
        if n.value:
            _call("qe_state_read", self.handle, which, _ptr(out), ctypes.byref(n), _stream(stream))
        return out


def probe_records(mode, records, accesses, sink, salt=0, stream=None):
    """Launches the random record probe over `records` (a device tensor of
    16-byte records, e.g. int32 [count, 4]): mode 0 reads, 1 reads and
    writes back `accesses` random records."""
    count = records.numel() * records.element_size() // 16
    _call("qe_probe_records", mode, _ptr(records), count, accesses, salt, _ptr(sink), _stream(stream))


def probe_lds(mode, workgroups, iters, sink, stream=None):
    """Launches the LDS bandwidth probe (mode 0 read, 1 write, 2 copy);
    returns the LDS bytes the launch moves."""
    b = ctypes.c_double(0)
    _call("qe_probe_lds", mode, workgroups, iters, _ptr(sink), ctypes.byref(b), _stream(stream))
    return b.value
