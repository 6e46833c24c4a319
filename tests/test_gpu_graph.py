"""Run modes of the batch driver (ttn_set_run_mode): static shapes (no host
read per centre move) reproduce the oracle like the dynamic mode, and the
whole op list captured once into a HIP graph and replayed gives records,
Kraus branches and log P bit-identical to the eager static-shape run at
every replay, with other GPU work and synchronisations between replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit  # noqa: E402
from oracle import statevector as sv  # noqa: E402


def _snap(res):
    return res.records.clone(), res.branches.clone(), res.logp.clone()


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("dtype,d,rounds,layout,rows", [("c128", 3, 3, None, 64),
                                                         ("c64", 5, 1, "optimized", 32)])
def test_graph_replays_equal_static_eager_runs(dtype, d, rounds, layout, rows):
    from paper_2511_05719_amd import TTNEngine
    circ = build_circuit(d, rounds, "srx+ad", leaf_of_qubit=layout)
    g = np.random.default_rng(14)
    th = torch.as_tensor(g.uniform(0.02, 0.3, (rows, circ.n_loc)), device="cuda")
    ga = torch.as_tensor(g.uniform(1e-3, 2e-2, (rows, circ.n_loc)), device="cuda")
    cut = 1e-15 if dtype == "c128" else 1e-10
    eng = TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=64, cutoff=cut, dtype=dtype, seed=3)
    ol = eng.upload(circ)
    offsets = (0, 4096)
    eng.run_mode("static")
    ref = {off: _snap(eng.run_circuit(ol, theta=th, gamma=ga, traj_offset=off)) for off in offsets}
    if dtype == "c128":
        # static shapes reproduce the oracle's records and branches exactly
        for off in offsets:
            o = sv.run(circ, th.cpu().numpy(), ga.cpu().numpy(), 3, np.arange(off, off + rows))
            assert np.array_equal(ref[off][0].cpu().numpy()[:, :circ.n_rec], o.records)
            assert np.array_equal(ref[off][1].cpu().numpy()[:, :circ.n_ad], o.branches)
            assert np.abs(ref[off][2].cpu().numpy() - o.logp).max() < 1e-9
    eng.run_mode("graph")
    out = eng.outputs(ol)
    for i, off in enumerate(offsets + offsets + offsets[:1]):
        res = eng.run_circuit(ol, theta=th, gamma=ga, traj_offset=off, out=out, stats=(i == 2))
        torch.cuda.synchronize()
        assert _same(_snap(res), ref[off]), (i, off)
        if i == 2:
            assert res.stats["flagged_rows"] == 0
        # other GPU work and a synchronisation between replays
        x = torch.arange(1 << 16, device="cuda", dtype=torch.float64)
        assert float((x * 2).sum().item()) == float((1 << 16) * ((1 << 16) - 1))
    captures, replays = eng.run_mode("graph")
    assert captures == 1 and replays == 5
    # new buffers: captured again
    eng.run_circuit(ol, theta=th, gamma=ga, traj_offset=0)
    assert eng.run_mode("graph")[0] == 2
    eng.close()


def test_dynamic_and_static_modes_agree_with_the_oracle():
    from paper_2511_05719_amd import TTNEngine
    circ = build_circuit(3, 2, "ad")
    rows = 128
    ref = sv.run(circ, 0.0, 0.02, 5, np.arange(rows))
    eng = TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=64, cutoff=1e-15, dtype="c128", seed=5)
    ol = eng.upload(circ)
    for mode in ("dynamic", "static", "dynamic"):
        eng.run_mode(mode)
        res = eng.run_circuit(ol, theta=0.0, gamma=0.02)
        assert np.array_equal(res.records.cpu().numpy(), ref.records), mode
        assert np.array_equal(res.branches.cpu().numpy(), ref.branches), mode
        assert np.abs(res.logp.cpu().numpy() - ref.logp).max() < 1e-9
    eng.close()


def test_graph_mode_rejects_profiling():
    from paper_2511_05719_amd import TTNEngine, TTNError
    circ = build_circuit(3, 1, "srx")
    eng = TTNEngine(circ.n_qubits, 4, circ.leaf_of_qubit, chi_max=64, cutoff=1e-15, dtype="c128", seed=0)
    ol = eng.upload(circ)
    eng.run_mode("graph")
    eng.profile(True)
    with pytest.raises(TTNError):
        eng.run_circuit(ol, theta=0.05, gamma=0.0)
    eng.profile(False)
    eng.run_circuit(ol, theta=0.05, gamma=0.0)
    with pytest.raises(ValueError):
        eng.run_mode("persistent")
    eng.close()
