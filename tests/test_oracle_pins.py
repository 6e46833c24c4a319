"""Pins of the FP64 oracle to facts fixed outside the oracle itself: published
known-answer vectors, closed forms of the paper's channels (Eq. 1-3, Eq. 9),
textbook special cases, the noiseless code circuit, and cross-checks between
independent methods (stabilizer tableau vs dense state vector; trajectory
averages vs the exact density matrix).  A dropped term, a wrong sign or a
transposed index in the oracle fails at least one of these."""
import os

import numpy as np
import pytest

from workload import build_circuit, custom_circuit, random_program
from oracle import channels, chp, closed_forms as cf, decoder, densitymatrix as dm, rng, stabrank
from oracle import statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MASK = (1 << 64) - 1


def _philox_ref(ctr, key):
    """Philox4x64-10 written from the SC'11 definition (test-side copy)."""
    M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
    W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
    c, k = list(ctr), list(key)
    for _ in range(10):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & MASK]
        k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
    return c


def test_philox_known_answers_and_stream_convention():
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert _philox_ref(v[0:4], v[4:6]) == v[6:10]
    # the oracle's stream: block j uses counter (j+1, 0, 0, 0), key (seed, traj)
    seed, tid = 11, 987654321
    w = rng.raw_words(seed, tid, 12)
    ref = sum((_philox_ref([j + 1, 0, 0, 0], [seed, tid]) for j in range(3)), [])
    assert [int(x) for x in w] == ref
    u = rng.uniforms(seed, [tid], 12)[0]
    assert np.array_equal(u, np.array([(x >> 11) * 2.0 ** -53 for x in ref]))


def _bloch(st, q):
    """Bloch vector of a single live qubit q (the register holds only q)."""
    psi = st.psi.reshape(st.T, 2)
    rho = np.einsum("ti,tj->tij", psi, psi.conj())
    return np.stack([np.real(np.einsum("tij,ji->t", rho, P)) for P in
                     (channels.X, channels.Y, channels.Z)], axis=1)


@pytest.mark.parametrize("theta", [0.05, 0.3, 1.1])
def test_srx_rotation_closed_form(theta):
    # exp(-i theta X/2) rotates the Bloch vector (0,0,1) to (0, -sin, cos)
    for k in range(1, 6):
        prog = [("init", 0, 0)] + [("srx", 0)] * k + [("meas", 0, 0)]
        circ = custom_circuit(1, prog)
        _, st = sv.run(circ, np.full(circ.n_loc, theta), 0.0, 0, [0], stop_after_op=k)
        b = _bloch(st, 0)[0]
        assert np.allclose(b, [0.0, -np.sin(k * theta), np.cos(k * theta)], atol=1e-14)
        assert abs(st.prob_one(0)[0] - cf.srx_flip_prob(theta, k)) < 1e-14


@pytest.mark.parametrize("theta", [0.05, 0.2])
def test_srx_twirl_closed_form(theta):
    pr = channels.pta_srx_probs(theta)
    assert np.allclose(pr, [np.cos(theta / 2) ** 2, np.sin(theta / 2) ** 2, 0, 0], atol=1e-15)
    for k in (1, 3, 7):
        prog = [("init", 0, 0)] + [("pauli", 0, 0)] * k + [("meas", 0, 0)]
        circ = custom_circuit(1, prog)
        p = dm.evolve(circ, np.full(circ.n_loc, theta), 0.0).diag_probs([0])
        assert abs(p[1] - cf.pta_srx_flip_prob(theta, k)) < 1e-14


@pytest.mark.parametrize("gamma", [1e-3, 1e-2, 0.3])
def test_ad_closed_forms(gamma):
    assert np.allclose(channels.pta_ad_probs(gamma), cf.pta_ad_probs(gamma), atol=1e-15)
    k0, k1 = channels.ad_kraus(gamma)
    assert np.allclose(k0.conj().T @ k0 + k1.conj().T @ k1, np.eye(2), atol=1e-15)
    for k in (1, 2, 5):
        # |1> (prepared by an X flip: twirled SRX at theta = pi) decays as (1-gamma)^k
        prog = [("init", 0, 0), ("pauli", 0, 0)] + [("ad", 0)] * k + [("meas", 0, 0)]
        circ = custom_circuit(1, prog)
        th = np.zeros(circ.n_loc); th[0] = np.pi
        ga = np.full(circ.n_loc, gamma); ga[0] = 0.0
        p = dm.evolve(circ, th, ga).diag_probs([0])
        assert abs(p[1] - cf.ad_excited_population(gamma, k)) < 1e-14
        # |+> keeps coherence (1-gamma)^(k/2)/2
        prog = [("init", 0, 1)] + [("ad", 0)] * k + [("meas", 0, 0)]
        circ = custom_circuit(1, prog)
        st = dm.evolve(circ, 0.0, np.full(circ.n_loc, gamma))
        assert abs(abs(st.rho.reshape(2, 2)[0, 1]) - cf.ad_plus_coherence(gamma, k)) < 1e-14
    # the jump probability of one trajectory step: gamma on |1>, gamma/2 on |+>
    circ = custom_circuit(1, [("init", 0, 0), ("pauli", 0, 0), ("ad", 0), ("meas", 0, 0)])
    r = sv.run(circ, np.array([np.pi, 0.0]), np.array([0.0, gamma]), 3, np.arange(4))
    jumped = r.branches[:, 0] == 1
    assert np.allclose(r.probs[jumped, 1], cf.ad_jump_prob_one(gamma))
    circ = custom_circuit(1, [("init", 0, 1), ("ad", 0), ("meas", 0, 0)])
    _, st = sv.run(circ, 0.0, np.full(1, gamma), 3, np.arange(1), stop_after_op=0)
    assert abs(gamma * st.prob_one(0)[0] - cf.ad_jump_prob_plus(gamma)) < 1e-15


@pytest.mark.parametrize("C", [1, 2])
def test_noiseless_d3_records(C):
    circ = build_circuit(3, C, "none")
    r = sv.run(circ, 0.0, 0.0, seed=1, traj_ids=np.arange(2000))
    P = circ.code.n_plaq
    assert np.allclose(r.logp, cf.noiseless_logp(P), atol=1e-12)
    assert not r.records[:, circ.zsyn_rec.ravel()].any()
    for rr in range(1, C):
        assert np.array_equal(r.records[:, circ.xsyn_rec[rr]], r.records[:, circ.xsyn_rec[0]])
    data = r.records[:, circ.data_rec]
    assert not decoder.decode_fail(circ.code.checks, data).any()
    assert not decoder.syndrome(circ.code.checks, data).any()
    assert len({tuple(x) for x in r.records}) == 2 ** (2 * P)


def test_noiseless_d5_stabilizer():
    circ = build_circuit(5, 2, "none")
    recs, _ = chp.run(circ, 0.0, 0.0, seed=2, traj_ids=np.arange(64))
    assert not recs[:, circ.zsyn_rec.ravel()].any()
    assert np.array_equal(recs[:, circ.xsyn_rec[1]], recs[:, circ.xsyn_rec[0]])
    assert not decoder.decode_fail(circ.code.checks, recs[:, circ.data_rec]).any()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_chp_matches_statevector_random_clifford(seed):
    g = np.random.default_rng(seed)
    nq = int(g.integers(4, 9))
    prog = random_program(nq, 12, g, noise=("pauli_srx", "pauli_ad"), measure_every=3)
    circ = custom_circuit(nq, prog)
    th = g.uniform(0.2, 1.2, circ.n_loc)
    ga = g.uniform(0.1, 0.6, circ.n_loc)
    r = sv.run(circ, th, ga, seed=seed, traj_ids=np.arange(200))
    recs, _ = chp.run(circ, th, ga, seed=seed, traj_ids=np.arange(200))
    assert np.array_equal(recs, r.records)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_stabilizer_rank_matches_svd(seed):
    g = np.random.default_rng(100 + seed)
    nq = 7
    prog = random_program(nq, 10, g, noise=("pauli_srx",))
    circ = custom_circuit(nq, prog)
    stop = int(np.nonzero(circ.ops[:, 0] == 5)[0][0]) - 1     # before the first measurement
    th = np.full(circ.n_loc, 0.7)
    _, tab = chp.run(circ, th, 0.0, seed, [0], stop_after_op=stop)
    _, st = sv.run(circ, th, 0.0, seed, [0], stop_after_op=stop)
    psi = st.full_state(nq)[0].reshape((2,) * nq)
    G = tab.stabilizers()
    for mask in range(1, 2 ** nq - 1):
        A = [q for q in range(nq) if mask >> q & 1]
        B = [q for q in range(nq) if not mask >> q & 1]
        m = np.transpose(psi, A + B).reshape(2 ** len(A), -1)
        s = np.linalg.svd(m, compute_uv=False)
        assert int((s > 1e-9).sum()) == stabrank.schmidt_rank(G, A)
        kept = s[s > 1e-9]
        assert np.allclose(kept, kept[0], rtol=1e-9)            # flat spectrum


def _within(k, n, p):
    lo, hi = decoder.wilson_interval(k, n)
    return lo <= p <= hi


def test_trajectory_average_matches_density_matrix_tiny():
    # 2 qubits, entangled, SRX + AD mixed: every outcome frequency inside its
    # 99.9% interval around the exact distribution
    prog = [("init", 0, 1), ("init", 1, 0), ("cnot", 0, 1), ("srxad", 0), ("srxad", 1),
            ("cnot", 1, 0), ("srxad", 0), ("ad", 1), ("meas", 0, 0), ("meas", 1, 0)]
    circ = custom_circuit(2, prog)
    th = np.array([0.4, 0.9, 0.3, 0.0])
    ga = np.array([0.2, 0.35, 0.5, 0.25])
    exact = dm.evolve(circ, th, ga).diag_probs([0, 1])
    Tn = 20000
    r = sv.run(circ, th, ga, seed=9, traj_ids=np.arange(Tn))
    idx = r.records[:, 0].astype(int) * 2 + r.records[:, 1]
    counts = np.bincount(idx, minlength=4)
    z = 3.29
    for k in range(4):
        lo, hi = decoder.wilson_interval(int(counts[k]), Tn, z)
        assert lo <= exact[k] <= hi


@pytest.mark.parametrize("channel,theta,gamma", [("ad", 0.0, 0.05), ("srx", 0.1, 0.0), ("pta_srx", 0.2, 0.0)])
def test_trajectory_pfail_matches_density_matrix_d3(channel, theta, gamma):
    circ = build_circuit(3, 1, channel)
    probs = dm.final_data_distribution(circ, np.full(circ.n_loc, theta), np.full(circ.n_loc, gamma))
    n = circ.code.n
    bits = ((np.arange(2 ** n)[:, None] >> (n - 1 - np.arange(n))) & 1)
    fail_of = decoder.decode_fail(circ.code.checks, bits)
    p_exact = float((probs * fail_of).sum())
    Tn = 3000
    r = sv.run(circ, theta, gamma, seed=4, traj_ids=np.arange(Tn))
    k = int(decoder.decode_fail(circ.code.checks, r.records[:, circ.data_rec]).sum())
    assert _within(k, Tn, p_exact), (k / Tn, p_exact)
    assert 0.005 < p_exact < 0.5


def test_forced_logp_matches_density_matrix():
    # P(full record) of a pure-state (SRX) circuit: the product of the
    # trajectory's conditional Born probabilities equals the trace of the
    # projected density matrix
    circ = build_circuit(3, 1, "srx")
    th = np.full(circ.n_loc, 0.4)
    r = sv.run(circ, th, 0.0, seed=5, traj_ids=np.arange(6))
    f = sv.run(circ, th, 0.0, seed=0, traj_ids=np.arange(6), forced_records=r.records)
    assert np.allclose(f.logp, r.logp, atol=1e-12)
    for t in range(3):
        st = dm.evolve(circ, th, 0.0, record=r.records[t], stop_before_final=False)
        assert abs(np.log(st.trace()) - r.logp[t]) < 1e-10


def test_decoder_corrects_low_weight_errors():
    from workload import build_color_code
    g = np.random.default_rng(0)
    for d in (3, 5):
        c = build_color_code(d)
        tab = decoder.leader_table(c.checks)
        t = (d - 1) // 2
        # random Z-bar = +1 codewords (sums of X-check rows: the noiseless final data)
        cw = (g.integers(0, 2, (32, c.n_plaq)) @ c.checks) % 2
        import itertools
        for w in range(t + 1):
            for sup in itertools.combinations(range(c.n), w):
                e = np.zeros(c.n, dtype=np.int64)
                e[list(sup)] = 1
                assert not decoder.decode_fail(c.checks, (cw + e) % 2, tab).any()
        # (a minimum-weight logical is not corrected:
        # test_decoder_fails_on_minimum_weight_logicals)


# ---------------------------------------------------------------- gradient ----
def test_gradient_closed_form_srx_measurement():
    # |0> -> SRX(t) -> Z measurement: P(1) = sin^2(t/2), P(0) = cos^2(t/2), so
    # d log P / dt = cot(t/2) for outcome 1 and -tan(t/2) for outcome 0
    from oracle import gradient
    circ = custom_circuit(1, [("init", 0, 0), ("srx", 0), ("meas", 0, 0)])
    for t in (0.3, 1.1, 2.0):
        for bit, want in ((1, 1.0 / np.tan(t / 2)), (0, -np.tan(t / 2))):
            lp, dth, dga = gradient.log_prob_grad(circ, [t], [0.0], [bit])
            assert abs(dth[0] - want) < 1e-12 * max(1.0, abs(want))
            assert abs(lp - np.log(np.sin(t / 2) ** 2 if bit else np.cos(t / 2) ** 2)) < 1e-12


def test_gradient_closed_form_amplitude_damping():
    # |0> -> SRX(t) -> AD(g) -> Z measurement: no jump then outcome 1 has
    # P = (1 - g) sin^2(t/2); a jump then outcome 0 has P = g sin^2(t/2)
    from oracle import gradient
    circ = custom_circuit(1, [("init", 0, 0), ("srxad", 0), ("meas", 0, 0)])
    t, g = 0.9, 0.07
    lp, dth, dga = gradient.log_prob_grad(circ, [t], [g], [1], [0])
    assert abs(lp - np.log((1 - g) * np.sin(t / 2) ** 2)) < 1e-12
    assert abs(dga[0] + 1.0 / (1.0 - g)) < 1e-10
    assert abs(dth[0] - 1.0 / np.tan(t / 2)) < 1e-10
    lp, dth, dga = gradient.log_prob_grad(circ, [t], [g], [0], [1])
    assert abs(lp - np.log(g * np.sin(t / 2) ** 2)) < 1e-12
    assert abs(dga[0] - 1.0 / g) < 1e-12
    assert abs(dth[0] - 1.0 / np.tan(t / 2)) < 1e-10


def test_gradient_matches_central_differences():
    # an independent route: central differences of the oracle's own log P
    from oracle import gradient
    from oracle import statevector as sv
    g = np.random.default_rng(5)
    nq = 5
    prog = [("init", q, int(g.integers(2))) for q in range(nq)]
    for _ in range(6):
        a, b = g.choice(nq, 2, replace=False)
        prog += [("cnot", int(a), int(b)), ("srxad", int(a)), ("srxad", int(b))]
        if g.random() < 0.4:
            q = int(g.integers(nq))
            prog += [("meas", q, int(g.integers(2))), ("init", q, 0), ("srxad", q)]
    prog += [("meas", q, 0) for q in range(nq)]
    circ = custom_circuit(nq, prog)
    th = g.uniform(0.05, 0.6, circ.n_loc)
    ga = g.uniform(0.01, 0.1, circ.n_loc)
    ref = sv.run(circ, th, ga, 3, np.arange(1))
    rec, br = ref.records[0], ref.branches[0]
    lp, dth, dga = gradient.log_prob_grad(circ, th, ga, rec, br)
    assert abs(lp - ref.logp[0]) < 1e-12
    h = 1e-6
    for l in range(circ.n_loc):
        tp, tm = th.copy(), th.copy()
        tp[l] += h
        tm[l] -= h
        fd = (gradient.log_prob(circ, tp, ga, rec[None], br[None])[0] -
              gradient.log_prob(circ, tm, ga, rec[None], br[None])[0]) / (2 * h)
        assert abs(fd - dth[l]) < 1e-6 * max(1.0, abs(dth[l])), (l, fd, dth[l])
        gp, gm = ga.copy(), ga.copy()
        gp[l] += h
        gm[l] -= h
        fd = (gradient.log_prob(circ, th, gp, rec[None], br[None])[0] -
              gradient.log_prob(circ, th, gm, rec[None], br[None])[0]) / (2 * h)
        assert abs(fd - dga[l]) < 1e-5 * max(1.0, abs(dga[l])), (l, fd, dga[l])


# ------------------------------------------------- binomial intervals ----
def test_wilson_interval_pins():
    # the interval every statistical comparison uses: fixed by its definition
    # (the p whose score statistic |k - n p| / sqrt(n p (1 - p)) equals z),
    # the normal quantile of a two-sided 99% level, k = 0 and mirror cases,
    # and its exact binomial coverage
    from scipy.stats import binom, norm
    z = 2.5758293035489004
    assert abs(z - norm.ppf(0.995)) < 1e-12
    for n in (1, 10, 1000):
        lo, hi = decoder.wilson_interval(0, n)
        assert lo == 0.0 and abs(hi - z * z / (n + z * z)) < 1e-15
    for n, k in ((50, 7), (1000, 13), (200, 100), (37, 36)):
        lo, hi = decoder.wilson_interval(k, n)
        lo2, hi2 = decoder.wilson_interval(n - k, n)
        assert abs(lo - (1 - hi2)) < 1e-14 and abs(hi - (1 - lo2)) < 1e-14
        for p in (lo, hi):
            if 0.0 < p < 1.0:
                assert abs((k - n * p) ** 2 - z * z * n * p * (1 - p)) < 1e-9 * n
        assert lo < k / n < hi
    n = 400
    for p in (0.01, 0.1, 0.5):
        cover = sum(binom.pmf(k, n, p) for k in range(n + 1)
                    if decoder.wilson_interval(k, n)[0] <= p <= decoder.wilson_interval(k, n)[1])
        assert 0.975 < cover < 0.9999, (p, cover)


def test_decoder_fails_on_minimum_weight_logicals():
    # X errors that commute with every Z check and flip Z-bar = Z^n (odd
    # weight) are logical operators; the lightest have weight d (the code
    # distance), and the decoder, seeing no syndrome, reports a failure
    import itertools
    from workload import build_color_code
    g = np.random.default_rng(3)
    for d in (3, 5):
        c = build_color_code(d)
        tab = decoder.leader_table(c.checks)
        cw = (g.integers(0, 2, (16, c.n_plaq)) @ c.checks) % 2
        found = 0
        for w in range(1, d + 1):
            for sup in itertools.combinations(range(c.n), w):
                e = np.zeros(c.n, dtype=np.int64)
                e[list(sup)] = 1
                if (c.checks @ e % 2).any() or w % 2 == 0:
                    continue
                assert w == d, f"logical of weight {w} < d = {d}"
                assert decoder.decode_fail(c.checks, (cw + e) % 2, tab).all()
                found += 1
        assert found > 0


# ------------------------------------------------ Trotterised AD reading ----
@pytest.mark.parametrize("mode", ["kraus", "trotter"])
def test_ad_nojump_branch_closed_form(mode):
    # one SRX(t) on |0>, one AD location, a Z measurement: forced no-jump
    # then outcome 1 has log P = log P(no jump) + log P(1 | no jump) of the
    # closed forms; the two readings differ at O(gamma^2)
    prog = [("init", 0, 0), ("srxad", 0), ("meas", 0, 0)]
    circ = custom_circuit(1, prog)
    for t, g in ((0.7, 0.2), (1.9, 0.05), (1.1, 1e-2)):
        pn, p1 = cf.ad_nojump_then_one(t, g, mode)
        r = sv.run(circ, [t], [g], 0, np.arange(1), forced_records=[[1]], forced_branches=[[0]], ad_mode=mode)
        assert abs(r.logp[0] - (np.log(pn) + np.log(p1))) < 1e-12
        assert abs(r.probs[0, 0] - pn) < 1e-14 and abs(r.probs[0, 1] - p1) < 1e-14
        other = cf.ad_nojump_then_one(t, g, "trotter" if mode == "kraus" else "kraus")[1]
        assert abs(other - p1) > 0.1 * g * g * np.sin(t / 2) ** 2 * np.cos(t / 2) ** 2
    # the no-jump gates themselves at gamma = 1e-2
    assert abs(channels.ad_trotter_nojump(1e-2)[1, 1].real - 0.9950125) < 1e-7
    assert abs(channels.ad_kraus(1e-2)[0][1, 1].real - 0.9949874) < 1e-7


def test_ad_trotter_jump_frequency_and_state():
    # the jump probability is gamma <n1> in both readings; sampled jump
    # frequencies fall inside their 99.9% intervals
    prog = [("init", 0, 0), ("srxad", 0), ("meas", 0, 0)]
    circ = custom_circuit(1, prog)
    t, g, Tn = 1.3, 0.3, 20000
    r = sv.run(circ, [t], [g], 5, np.arange(Tn), ad_mode="trotter")
    k = int(r.branches[:, 0].sum())
    lo, hi = decoder.wilson_interval(k, Tn, 3.29)
    assert lo <= g * np.sin(t / 2) ** 2 <= hi
    # after a jump the qubit is |0>; after no jump it reads 1 with the
    # Trotter closed form
    assert not r.records[r.branches[:, 0] == 1, 0].any()
    nj = r.branches[:, 0] == 0
    k1 = int(r.records[nj, 0].sum())
    lo, hi = decoder.wilson_interval(k1, int(nj.sum()), 3.29)
    assert lo <= cf.ad_nojump_then_one(t, g, "trotter")[1] <= hi
