"""Dense definition of a circuit unitary by Kronecker products (numpy, fp64).

Test infrastructure only.  This is the textbook construction, written
independently of the per-gate oracle so that each can pin the other:
every gate is expanded to the full register width with Kronecker products in
the order of Eq. 1 (the first factor is wire 0, the most significant bit of a
basis index), a controlled gate as |0><0| (x) I + |1><1| (x) U placed on its
wires, and the circuit is the product of the expanded gates, the gate listed
first applied first.  Only meant for n <= 4.

Ising gates (kinds 7-10) take an angle theta in radians.  The rotations are
the matrices of Eqs. 3-5 expanded like any single-qubit gate; the
interaction on wires (a, b) is built the way Sec. IV-A describes its
templates: the full-width diagonal of +-1 entries (Z on wires a and b, the
identity elsewhere) is exponentiated element by element, J = exp(-i theta/2
Z_a Z_b), which is Eq. 6 read with the exponent i theta.
"""
import numpy as np

I2 = np.eye(2, dtype=complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
V = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]])
VDG = V.conj().T
H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
TG = np.diag([1, np.exp(1j * np.pi / 4)])
P0 = np.diag([1, 0]).astype(complex)
P1 = np.diag([0, 1]).astype(complex)

Z = np.diag([1.0, -1.0]).astype(complex)

SINGLE = {1: X, 5: H, 6: TG}


def rotation(kind, theta):
    """Eqs. 3-5."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    if kind == 7:
        return np.array([[c, -1j * s], [-1j * s, c]])
    if kind == 8:
        return np.array([[c, -s], [s, c]], dtype=complex)
    return np.array([[np.exp(-1j * theta / 2), 0], [0, np.exp(1j * theta / 2)]])


def template(n, a, b):
    """The +-1 diagonal of the interaction template on wires (a, b)."""
    return np.real(np.diag(kron_all([Z if w in (a, b) else I2 for w in range(n)])))
CONTROLLED = {2: X, 3: V, 4: VDG}


def kron_all(factors):
    out = np.array([[1.0 + 0j]])
    for f in factors:
        out = np.kron(out, f)
    return out


def expand(n, d, theta=0.0):
    """Full 2^n x 2^n matrix of descriptor d (theta: angle of an Ising gate)."""
    kind, t, c = d & 15, (d >> 4) & 15, (d >> 8) & 15
    if kind == 0:
        return np.eye(1 << n, dtype=complex)
    if kind in (7, 8, 9):
        R = rotation(kind, theta)
        return kron_all([R if w == t else I2 for w in range(n)])
    if kind == 10:
        return np.diag(np.exp(-0.5j * theta * template(n, t, c)))
    if kind in SINGLE:
        return kron_all([SINGLE[kind] if w == t else I2 for w in range(n)])
    U = CONTROLLED[kind]
    off = kron_all([P0 if w == c else I2 for w in range(n)])
    on = kron_all([P1 if w == c else (U if w == t else I2) for w in range(n)])
    return off + on


def unitary(n, gates, thetas=None):
    """thetas: angles in radians, one per gate (Ising gates only)."""
    S = np.eye(1 << n, dtype=complex)
    for k, d in enumerate(gates):
        S = expand(n, int(d), 0.0 if thetas is None else float(thetas[k])) @ S
    return S


def fitness_eq11(n, S, T):
    """Eq. 11 as printed: 1 - sqrt((size - |tr(S^dagger T)|) / size)."""
    size = 2 ** n
    tr = np.trace(S.conj().T @ T)
    return 1.0 - np.sqrt(max(0.0, (size - abs(tr)) / size))
