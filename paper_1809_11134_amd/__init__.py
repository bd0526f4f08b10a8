"""MI355X (gfx950) implementation of the circuit-fitness hot path of the
Quantum Encoded Quantum Evolutionary Algorithm (Krylov & Lukac,
arXiv:1809.11134): batched Eq. 11 fitness of library-gate circuits, circuit
construction by sampling a qubit/qutrit encoding, and the QEQEA / GA update
loop, all in hand-written HIP kernels behind the C ABI of include/qe.h.

``qe`` is the Python binding (ctypes + torch device memory and streams),
``inputs`` the seeded synthetic workloads, ``build`` the hipcc build."""
