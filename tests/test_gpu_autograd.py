"""log P(record) through torch.autograd (paper_2511_05719_amd.autograd), whose
backward is the library's hand-written adjoint: gradients against the
oracle's exact derivatives (oracle/gradient.py) at d=3, the tied scalar
gradient against the sum over locations, and torch's own finite-difference
gradcheck on a small circuit (complex128, untruncated)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit, custom_circuit  # noqa: E402
from oracle import gradient  # noqa: E402
from oracle import statevector as sv  # noqa: E402

CUT_EXACT = 1e-15


def _engine(circ, rows, dtype="c128", seed=0):
    from paper_2511_05719_amd import TTNEngine
    return TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=64,
                     cutoff=CUT_EXACT if dtype == "c128" else 1e-10, dtype=dtype, seed=seed)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-6), ("c64", 1e-3)])
def test_autograd_matches_oracle_gradient_d3(dtype, tol):
    # d=3 colour code, 1 round, SRX + AD at every location, per-row and
    # per-location parameters: d(sum_rows w_r log P_r)/d theta[r, l] = w_r *
    # the oracle's d log P_r / d theta_l (and likewise for gamma)
    from paper_2511_05719_amd import log_prob
    circ = build_circuit(3, 1, "srx+ad")
    rows = 6
    g = np.random.default_rng(12)
    th0 = g.uniform(0.05, 0.4, (rows, circ.n_loc))
    ga0 = g.uniform(0.005, 0.05, (rows, circ.n_loc))
    ref = sv.run(circ, th0, ga0, 3, np.arange(rows))
    eng = _engine(circ, rows, dtype)
    ol = eng.upload(circ)
    th = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    ga = torch.tensor(ga0, dtype=torch.float64, requires_grad=True)
    lp = log_prob(eng, ol, ref.records, ref.branches, th, ga)
    w = torch.linspace(0.5, 2.0, rows, dtype=torch.float64, device=lp.device)
    (w * lp).sum().backward()
    wn = w.cpu().numpy()
    for r in range(rows):
        l0, dt0, dg0 = gradient.log_prob_grad(circ, th0[r], ga0[r], ref.records[r], ref.branches[r])
        assert abs(lp[r].item() - l0) < (1e-7 if dtype == "c128" else 1e-4)
        et = np.abs(th.grad[r].numpy() - wn[r] * dt0) / np.maximum(1.0, np.abs(wn[r] * dt0))
        eg = np.abs(ga.grad[r].numpy() - wn[r] * dg0) / np.maximum(1.0, np.abs(wn[r] * dg0))
        assert et.max() < tol and eg.max() < tol, (r, et.max(), eg.max())
    eng.close()


def test_autograd_tied_parameters_sum_over_locations():
    # one theta and one gamma tied over every location (scalars): the
    # gradient is the sum of the per-location derivatives over rows and
    # locations
    from paper_2511_05719_amd import log_prob
    circ = build_circuit(3, 1, "srx+ad")
    rows = 4
    ref = sv.run(circ, 0.2, 0.02, 5, np.arange(rows))
    eng = _engine(circ, rows)
    ol = eng.upload(circ)
    th = torch.tensor(0.2, dtype=torch.float64, requires_grad=True)
    ga = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    log_prob(eng, ol, ref.records, ref.branches, th, ga).sum().backward()
    st = sg = 0.0
    for r in range(rows):
        _, dt0, dg0 = gradient.log_prob_grad(circ, np.full(circ.n_loc, 0.2), np.full(circ.n_loc, 0.02),
                                             ref.records[r], ref.branches[r])
        st += dt0.sum()
        sg += dg0.sum()
    assert abs(th.grad.item() - st) < 1e-6 * max(1.0, abs(st))
    assert abs(ga.grad.item() - sg) < 1e-6 * max(1.0, abs(sg))
    eng.close()


def test_autograd_gradcheck_small_circuit():
    # torch's central differences of the forward pass against the backward
    from paper_2511_05719_amd import log_prob
    nq = 4
    prog = [("init", 0, 1), ("init", 1, 0), ("init", 2, 1), ("init", 3, 0),
            ("cnot", 0, 1), ("srxad", 0), ("srxad", 1), ("cnot", 2, 3), ("srxad", 2), ("srxad", 3),
            ("cnot", 1, 2), ("srxad", 1), ("srxad", 2), ("meas", 1, 0), ("init", 1, 0), ("srxad", 1),
            ("cnot", 0, 3), ("srxad", 0), ("srxad", 3)] + [("meas", q, 0) for q in range(nq)]
    circ = custom_circuit(nq, prog)
    rows = 2
    g = np.random.default_rng(4)
    th0 = g.uniform(0.2, 0.8, circ.n_loc)
    ga0 = g.uniform(0.05, 0.2, circ.n_loc)
    ref = sv.run(circ, th0, ga0, 8, np.arange(rows))
    eng = _engine(circ, rows)
    ol = eng.upload(circ)
    th = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    ga = torch.tensor(ga0, dtype=torch.float64, requires_grad=True)

    def f(t, a):
        return log_prob(eng, ol, ref.records, ref.branches, t, a)

    assert torch.autograd.gradcheck(f, (th, ga), eps=1e-6, atol=1e-5, rtol=1e-4)
    eng.close()


def test_autograd_without_grad_runs_the_forward_only():
    from paper_2511_05719_amd import log_prob
    circ = build_circuit(3, 1, "srx")
    rows = 3
    ref = sv.run(circ, 0.1, 0.0, 2, np.arange(rows))
    eng = _engine(circ, rows)
    ol = eng.upload(circ)
    with torch.no_grad():
        lp = log_prob(eng, ol, ref.records, None, torch.tensor(0.1, dtype=torch.float64), 0.0)
    assert not lp.requires_grad
    assert np.abs(lp.cpu().numpy() - ref.logp).max() < 1e-9
    eng.close()
