"""Dense definition of a circuit unitary by Kronecker products (numpy, fp64).

Test infrastructure only.  This is the textbook construction, written
independently of the per-gate oracle so that each can pin the other:
every gate is expanded to the full register width with Kronecker products in
the order of Eq. 1 (the first factor is wire 0, the most significant bit of a
basis index), a controlled gate as |0><0| (x) I + |1><1| (x) U placed on its
wires, and the circuit is the product of the expanded gates, the gate listed
first applied first.  Only meant for n <= 4.
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

SINGLE = {1: X, 5: H, 6: TG}
CONTROLLED = {2: X, 3: V, 4: VDG}


def kron_all(factors):
    out = np.array([[1.0 + 0j]])
    for f in factors:
        out = np.kron(out, f)
    return out


def expand(n, d):
    """Full 2^n x 2^n matrix of descriptor d."""
    kind, t, c = d & 15, (d >> 4) & 15, (d >> 8) & 15
    if kind == 0:
        return np.eye(1 << n, dtype=complex)
    if kind in SINGLE:
        return kron_all([SINGLE[kind] if w == t else I2 for w in range(n)])
    U = CONTROLLED[kind]
    off = kron_all([P0 if w == c else I2 for w in range(n)])
    on = kron_all([P1 if w == c else (U if w == t else I2) for w in range(n)])
    return off + on


def unitary(n, gates):
    S = np.eye(1 << n, dtype=complex)
    for d in gates:
        S = expand(n, int(d)) @ S
    return S


def fitness_eq11(n, S, T):
    """Eq. 11 as printed: 1 - sqrt((size - |tr(S^dagger T)|) / size)."""
    size = 2 ** n
    tr = np.trace(S.conj().T @ T)
    return 1.0 - np.sqrt(max(0.0, (size - abs(tr)) / size))
