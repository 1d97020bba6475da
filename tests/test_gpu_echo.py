"""The Loschmidt echo of Sec. 4.2 on the GPU: a periodic Heisenberg ring, with and without
the double-quantum terms S^x S^x - S^y S^y up to the third neighbour, from the random
superposition |up>_0 (x) random phases, evolved n steps forward and n steps with -dt.

U4 is palindromic, so the backward run is the exact inverse up to rounding: the state must
come back (|1 - M_LE| and the distance at the rounding level), the forward state must equal
the oracle's to 1e-10 relative L2 (complex128), and the echo state the oracle's echo state.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1305_0036_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_0036_amd import tsspin
    return tsspin


@pytest.mark.parametrize("dq", [False, True])
def test_echo_ring_matches_oracle(dq):
    ts = _dev()
    n, steps = 12, 40
    w = W.echo_ring(n=n, double_quantum=dq)
    print("[case] echo ring n=12 dq=", dq, flush=True)
    H = ts.Hamiltonian(w.n, w.bonds, w.fields)
    Ho = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    x0 = torch.from_numpy(w.psi0).cuda()
    x = x0.clone()
    H.evolve(x, w.dt, steps, 4)
    fwd = oracle.evolve(Ho, w.psi0, w.dt, steps, 4)
    got = x.cpu().numpy()
    assert np.linalg.norm(got - fwd) / np.linalg.norm(fwd) < 1e-10
    H.evolve(x, -w.dt, steps, 4)
    back = oracle.evolve(Ho, fwd, -w.dt, steps, 4)
    got = x.cpu().numpy()
    assert np.linalg.norm(got - back) < 1e-10
    assert np.linalg.norm(got - w.psi0) < 1e-11
    ov = H.expect(x, [("overlap", x0)])[0]
    m_le = abs(ov) ** 2
    assert abs(1.0 - m_le) < 1e-12
    # the library's overlap is the plain inner product
    assert abs(ov - np.vdot(w.psi0, got)) < 1e-13


def test_echo_ring_complex64_and_records():
    """complex64: the echo returns to 1e-5; the overlap recorded by ts_evolve between two
    evolved vectors equals the one computed afterwards."""
    ts = _dev()
    w = W.echo_ring(n=14, double_quantum=True)
    H = ts.Hamiltonian(w.n, w.bonds, w.fields)
    x0 = torch.from_numpy(w.psi0).to(torch.complex64).cuda()
    x = x0.clone()
    H.evolve(x, w.dt, 30, 4)
    H.evolve(x, -w.dt, 30, 4)
    m_le = abs(H.expect(x, [("overlap", x0)])[0]) ** 2
    assert abs(1.0 - m_le) < 1e-5
    a = torch.from_numpy(w.psi0).cuda()
    b = a.clone()
    rec = H.evolve([a, b], w.dt, 4, 4, record=[("overlap", 0, 1), ("norm", 1)], rec_every=2).cpu().numpy()
    assert rec.shape == (3, 3)
    assert np.allclose(rec[:, 0], 1.0, atol=1e-13) and np.allclose(rec[:, 1], 0.0, atol=1e-13)
    assert np.allclose(rec[:, 2], 1.0, atol=1e-13)
