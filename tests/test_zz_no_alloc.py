"""qe_eval_fitness_noalloc (the evaluation entry point for callers that cannot
allocate: its workspace is a fixed array inside the library) against
qe_eval_fitness_ws with a caller workspace, through the C ABI: two calls in a
row, the second with a smaller batch, then a uniform batch; and the size
limit, checked on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def mixed_batch(rng, oracle, dev, B, lib=inputs.LIB_HT_NCV):
    nq = rng.integers(1, 7, size=B).astype(np.int8)
    lens = rng.integers(0, 70, size=B)
    goff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    gates = np.concatenate([inputs.random_circuits(rng, 1, int(n), int(L), lib)[0]
                            for n, L in zip(nq, lens)] + [np.zeros(0, np.uint16)]).astype(np.uint16)
    mats, toff, o = [], [], 0
    for n in nq:
        T = oracle.unitary(int(n), inputs.random_target_gates(rng, int(n), 6, lib))
        mats.append(T.ravel())
        toff.append(o)
        o += T.size
    T = np.concatenate(mats)
    toff = np.array(toff, np.int64)
    d = dict(nq=torch.from_numpy(nq).to(dev), goff=torch.from_numpy(goff).to(dev),
             toff=torch.from_numpy(toff).to(dev))
    b, keep, _ = qe.make_batch(torch.from_numpy(gates.view(np.int16)).to(dev),
                               torch.from_numpy(T).to(dev).to(torch.complex64), target_stride=None, **d)
    ref = oracle.eval_batch(nq, goff, gates, toff, T)[:, 0]
    return b, keep, ref


def run_both(b, B, dev):
    out = []
    for name in ("qe_eval_fitness_noalloc", "qe_eval_fitness_ws"):
        f = torch.full((B,), -7.0, dtype=torch.float32, device=dev)
        g = torch.full((B,), -7.0, dtype=torch.float32, device=dev)
        d = torch.full((B,), -7.0, dtype=torch.float32, device=dev)
        if name == "qe_eval_fitness_noalloc":
            qe._call(name, ctypes.byref(b), qe.PATH_FP32, qe._ptr(f), qe._ptr(g), qe._ptr(d), qe._stream(None))
        else:
            ws = qe.eval_workspace(B, dev)
            qe._call(name, ctypes.byref(b), qe.PATH_FP32, qe._ptr(f), qe._ptr(g), qe._ptr(d), qe._ptr(ws),
                     ws.numel() * 4, qe._stream(None))
        out.append((f, g, d))
    torch.cuda.synchronize()
    return out


def test_noalloc_matches_workspace_entry(dev, oracle):
    rng = np.random.default_rng(4242)
    for B in (3000, 700):            # the second call with a smaller batch
        b, keep, ref = mixed_batch(rng, oracle, dev, B)
        (fa, ga, da), (fw, gw, dw) = run_both(b, B, dev)
        assert torch.equal(fa, fw) and torch.equal(ga, gw) and torch.equal(da, dw), B
        assert np.abs(fa.cpu().numpy().astype(np.float64) - ref).max() <= 1e-5, B
    # a uniform batch needs no scratch; the result is the usual one
    n, L, B = 5, 24, 96
    gates = inputs.random_circuits(rng, B, n, L, inputs.LIB_HT_NCV)
    T = oracle.unitary(n, inputs.random_target_gates(rng, n, 10, inputs.LIB_HT_NCV))
    b, keep, _ = qe.make_batch(torch.from_numpy(gates.view(np.int16)).to(dev),
                               torch.from_numpy(T).to(dev).to(torch.complex64), n=n, L=L, target_stride=0)
    (fa, _, _), (fw, _, _) = run_both(b, B, dev)
    assert torch.equal(fa, fw)
    assert qe.device_errors() == 0


def test_noalloc_rejects_too_many_circuits(dev):
    b = qe.Batch()
    b.num_circuits = 262145          # QE_NOALLOC_MAX_CIRCUITS + 1, mixed widths
    b.uniform_n = 0
    with pytest.raises(qe.QeError) as e:
        qe._call("qe_eval_fitness_noalloc", ctypes.byref(b), qe.PATH_FP32, None, None, None, qe._stream(None))
    assert e.value.status == qe.QE_ERR_INVALID
    assert "QE_NOALLOC_MAX_CIRCUITS" in str(e.value)
