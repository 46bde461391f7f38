"""Pins of the CPU oracle to facts that do not come from the oracle itself:
published known-answer vectors, numbers printed in the paper, closed forms,
brute force over every state of tiny systems, and exact invariants.  Each
test names the passage it follows."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as WL

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- Philox ----

def test_philox_known_answers():
    """Known-answer vectors published with the Random123 library of Salmon et
    al. (SC'11) for Philox4x32-10."""
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        assert oracle.philox4x32_10(ctr, key).tolist() == want


def _half(block, j):
    return (int(block[j >> 1]) >> (16 * (j & 1))) & 0xFFFF


def test_sample_counter_layout_and_thresholds():
    """With K = 16 uniform states the thresholds are s * 2^28, so the state of
    component i of sample h is the top nibble of its word, i.e. of the high
    16-bit half: half (i mod 8) (word (i mod 8) div 2, low half first) of the
    block with counter (i div 8, low32(h), high32(h), stream) and key
    (low32(seed), high32(seed))."""
    K, n = 16, 19
    p = np.full((n, K), 1.0 / K)
    seed, stream = 0xDEADBEEF12345678, 9
    first = (1 << 32) - 3
    x = oracle.sample(p, seed, stream, first, 6)
    for hh in range(6):
        h = first + hh
        for i in range(n):
            ctr = [i >> 3, h & 0xFFFFFFFF, h >> 32, stream]
            key = [seed & 0xFFFFFFFF, seed >> 32]
            assert x[hh, i] == _half(oracle.philox4x32_10(ctr, key), i & 7) >> 12


# ------------------------------------------------------------- thresholds ----

def _word_of_sample0_component(i):
    """The full 32-bit word of component i of sample 0 (seed 0, stream 0):
    high half from counter (i div 8, 0, 0, 0), low half from the same counter
    with bit 31 of its first word set."""
    hi = oracle.philox4x32_10([i >> 3, 0, 0, 0], [0, 0])
    lo = oracle.philox4x32_10([(i >> 3) | 0x80000000, 0, 0, 0], [0, 0])
    return (_half(hi, i & 7) << 16) | _half(lo, i & 7)


def test_state_flips_exactly_at_the_threshold():
    """x = 1 iff u >= C.  Component 0 of sample 0 under seed 0, stream 0 has
    high half 0xE8D5, the low half of the first Random123 known-answer word
    0x6627E8D5; a failure probability of exactly u / 2^32 puts the threshold
    on u (state 1), one more unit above it (state 0).  The thresholds share
    u's high half, so only the low half decides."""
    word = _word_of_sample0_component(0)
    assert word >> 16 == 0xE8D5
    for c, want in ((word, 1), (word + 1, 0), (word - 1, 1)):
        q = c / 4294967296.0          # exact in fp64
        p = np.array([[q, 1.0 - q]])
        assert int(oracle.thresholds(p)[0, 0]) == c
        assert int(oracle.sample(p, 0, 0, 0, 1)[0, 0]) == want
    # The same for a component in the second group of eight, position 5.
    word = _word_of_sample0_component(13)
    n = 14
    for c, want in ((word, 1), (word + 1, 0)):
        q = c / 4294967296.0
        p = np.tile([[0.5, 0.5]], (n, 1))
        p[13] = [q, 1.0 - q]
        assert int(oracle.sample(p, 0, 0, 0, 1)[0, 13]) == want


def test_thresholds_exact_edges():
    two32 = 1 << 32
    p_surv = np.array([0.0, 1.0, 0.5, 2.0 ** -32, 1.0 - 2.0 ** -53])
    C = oracle.thresholds(oracle.state_probs_binary(p_surv))[:, 0]
    # P(x = 1) = (2^32 - C) / 2^32 exactly for these dyadic probabilities.
    assert C.tolist() == [two32, 0, two32 // 2, two32 - 1, 0]


def test_sample_frequencies_within_5_sigma():
    rng = np.random.default_rng(3)
    n, K, N = 24, 3, 200_000
    p = rng.dirichlet([2.0, 1.0, 1.0], size=n)
    x = oracle.sample(p, 42, 0, 0, N)
    for s in range(K):
        freq = (x == s).mean(axis=0)
        sigma = np.sqrt(p[:, s] * (1 - p[:, s]) / N)
        assert np.all(np.abs(freq - p[:, s]) <= 5 * sigma + 1e-12)


def test_sample_ranges_and_threads_agree():
    p = oracle.state_probs_binary(np.linspace(0.1, 0.9, 40))
    full = oracle.sample(p, 5, 1, 0, 3000)
    part = oracle.sample(p, 5, 1, 1000, 2000)
    np.testing.assert_array_equal(full[1000:], part)
    idx = np.array([0, 17, 2999, 1000], dtype=np.uint64)
    np.testing.assert_array_equal(oracle.sample_at(p, 5, 1, idx), full[idx.astype(int)])
    t = oracle.get_threads()
    oracle.set_threads(1)
    single = oracle.sample(p, 5, 1, 0, 3000)
    oracle.set_threads(t)
    np.testing.assert_array_equal(full, single)


# ------------------------------------------------ encoding / classification --

def _golden_worked():
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "worked_example_2x5.txt"))
             if ln.strip() and not ln.startswith("#")]
    data = {"lower": [], "upper": [], "sample": [], "unclassified": [], "matrix": {},
            "phi_zero": [], "phi_one": [], "boundary_from": [], "boundary_result": []}
    k = 0
    while k < len(lines):
        tok = lines[k].split()
        if tok[0] == "M":
            data["M"] = int(tok[1])
            k += 1
        elif tok[0] == "matrix":
            key = (tok[1], int(tok[2]), int(tok[3]))
            rows = [list(map(int, lines[k + 1].split())), list(map(int, lines[k + 2].split()))]
            data["matrix"][key] = np.array(rows, dtype=np.uint8)
            k += 3
        else:
            data[tok[0]].append((int(tok[1]), int(tok[2])))
            k += 1
    return data


def test_worked_example_encodings_match_printed_matrices():
    """Section 3.2: the printed matrices of x1^L = (1,2), x1^U = (1,4),
    x2^U = (4,0) and the samples (3,0), (4,4)."""
    d = _golden_worked()
    M = d["M"]
    for r in d["lower"]:
        _, _, R = oracle.paper_violation([0, 0], r, M, side=0)
        np.testing.assert_array_equal(R, d["matrix"][("lower",) + r])
    for r in d["upper"]:
        _, _, R = oracle.paper_violation([0, 0], r, M, side=1)
        np.testing.assert_array_equal(R, d["matrix"][("upper",) + r])
    for x in d["sample"]:
        _, H, _ = oracle.paper_violation(x, [0, 0], M, side=0)
        np.testing.assert_array_equal(H, d["matrix"][("sample",) + x])


def test_violation_zero_iff_componentwise_order():
    """Section 3.3.2: V(h, r) = 0 exactly when the sample is dominated; the
    oracle's classification (componentwise order of section 2.2) must agree
    with the paper's matrix formula on all 25 states of the worked example,
    and (2,0) must be unclassified (section 3.4, fig. x1x2_find_ref)."""
    d = _golden_worked()
    M = d["M"]
    lower = np.array(d["lower"], dtype=np.uint8)
    upper = np.array(d["upper"], dtype=np.uint8)
    states = np.array([(a, b) for a in range(M) for b in range(M)], dtype=np.uint8)
    flags, mL, mU = oracle.classify(lower, upper, states, mode=1)
    for k, x in enumerate(states):
        vL = [oracle.paper_violation(x, r, M, 0)[0] for r in lower]
        vU = [oracle.paper_violation(x, r, M, 1)[0] for r in upper]
        assert mL[k] == sum(v == 0 for v in vL)
        assert mU[k] == sum(v == 0 for v in vU)
    look = {tuple(s): f for s, f in zip(states.tolist(), flags)}
    assert look[(4, 4)] == 2             # above x1^U and x2^U
    assert look[(3, 0)] == 0
    for x in d["unclassified"]:
        assert look[x] == 0
    # V rows of the two highlighted samples.
    assert [oracle.paper_violation((3, 0), r, M, 0)[0] for r in lower] == [1]
    assert [oracle.paper_violation((3, 0), r, M, 1)[0] for r in upper] == [1, 1]
    assert [oracle.paper_violation((4, 4), r, M, 0)[0] for r in lower] == [2]
    assert [oracle.paper_violation((4, 4), r, M, 1)[0] for r in upper] == [0, 0]


def test_label_mode_lower_precedence():
    """Algorithm 1: a sample dominated on both sides is lower-classified; the
    label mode then does not examine the upper set."""
    lower = np.array([[1, 1]], dtype=np.uint8)
    upper = np.array([[0, 0]], dtype=np.uint8)
    x = np.array([[0, 1], [1, 1]], dtype=np.uint8)
    fl, _, _ = oracle.classify(lower, upper, x, mode=0)
    fc, mL, mU = oracle.classify(lower, upper, x, mode=1)
    assert fl.tolist() == [1, 1]
    assert fc.tolist() == [3, 3]
    cnt = oracle.counts(fc)
    assert cnt[0] == 2 and cnt[1] == 0 and cnt[3] == 2


# ------------------------------------------------------ printed numbers ----

def _golden_numbers():
    out = {}
    for ln in open(os.path.join(GOLDEN, "paper_numbers.txt")):
        if ln.strip() and not ln.startswith("#"):
            tok = ln.split()
            out[tok[0]] = [float(v) for v in tok[1:]]
    return out


def test_toy_state_probability():
    """Section 2.2: P(x3) = 0.1 * 0.9^5, printed as 0.0590."""
    g = _golden_numbers()
    p = oracle.state_probs_binary(np.full(6, 0.9))
    x3 = np.array([0, 1, 1, 1, 1, 1], dtype=np.uint8)
    assert round(oracle.state_prob(p, x3), 4) == g["toy_state_prob"][0]


def test_worked_counts_to_probabilities():
    """Section 3.3.1: |I^L| = 3, |I^U| = 4, |I^u| = 3 of H = 10 samples give
    0.3 / 0.4 / 0.3."""
    g = _golden_numbers()
    nL, nU, nu = (int(v) for v in g["worked_counts"])
    est = oracle.estimate([nL, nU, nu, 0, 0, 10], has_Y=False)
    assert est[:3].tolist() == g["worked_probs"]


def test_pmf_by_differences():
    """Section 3.5 and tab. rsr_multistate: P(S = m') from cumulative values."""
    g = _golden_numbers()
    pmf = oracle.pmf_from_cdf(g["multistate_cdf"])
    assert [float(f"{v:.3g}") for v in pmf] == g["multistate_pmf"]


def test_estimator_closed_forms():
    """Section 3.3.1: p = |I| / H and delta = sqrt((1 - p) / (H p))."""
    est = oracle.estimate([10, 30, 60, 0, 20, 100])
    assert est[3] == 0.5
    assert est[4] == math.sqrt(0.5 * 0.5 / 100)
    assert est[5] == math.sqrt(0.5 / (100 * 0.5))
    est = oracle.estimate([70, 20, 10, 0, 5, 100])
    assert est[3] == 0.25
    assert abs(est[4] - math.sqrt(0.25 * 0.75 / 100)) < 1e-15
    assert abs(est[5] - math.sqrt(0.75 / (100 * 0.25))) < 1e-15
    zero = oracle.estimate([100, 0, 0, 0, 0, 100])
    assert zero[3] == 0.0 and math.isinf(zero[5])


# ---------------------------------------------- brute force and closed forms --

def _graph(n_nodes, edges, s, t):
    e = np.array(edges, dtype=np.int32)
    return {"n_nodes": n_nodes, "edge_u": e[:, 0].copy(), "edge_v": e[:, 1].copy(),
            "source": s, "sink": t}


def _bridge():
    # s=0, t=3; edges 0:(0,1) 1:(0,2) 2:(1,3) 3:(2,3) 4:(1,2) - the Wheatstone bridge.
    return _graph(4, [(0, 1), (0, 2), (1, 3), (2, 3), (1, 2)], 0, 3)


def _bridge_closed_form(p):
    p1, p2, p3, p4, p5 = p
    with5 = (1 - (1 - p1) * (1 - p2)) * (1 - (1 - p3) * (1 - p4))
    without5 = 1 - (1 - p1 * p3) * (1 - p2 * p4)
    return p5 * with5 + (1 - p5) * without5


def test_closed_forms_series_parallel_bridge():
    rng = np.random.default_rng(8)
    n = 7
    p = rng.uniform(0.3, 0.95, n)
    series = _graph(n + 1, [(i, i + 1) for i in range(n)], 0, n)
    parallel = _graph(2, [(0, 1)] * n, 0, 1)
    for g, want in [(series, np.prod(p)), (parallel, 1 - np.prod(1 - p))]:
        P, _ = oracle.exact(oracle.state_probs_binary(p), oracle.phi_table_st(g), want_grad=False)
        assert abs(P - want) < 1e-14
    pb = rng.uniform(0.3, 0.95, 5)
    P, _ = oracle.exact(oracle.state_probs_binary(pb), oracle.phi_table_st(_bridge()),
                        want_grad=False)
    assert abs(P - _bridge_closed_form(pb)) < 1e-14


def test_closed_forms_multistate_levels():
    """Bottleneck levels of 3-state series and parallel systems: S >= k needs
    every (series) or some (parallel) edge in a state >= k."""
    rng = np.random.default_rng(9)
    n = 6
    p = rng.dirichlet([1.0, 1.5, 2.0], size=n)
    series = _graph(n + 1, [(i, i + 1) for i in range(n)], 0, n)
    parallel = _graph(2, [(0, 1)] * n, 0, 1)
    for level in (1, 2):
        ge = p[:, level:].sum(axis=1)
        for g, want in [(series, np.prod(ge)), (parallel, 1 - np.prod(1 - ge))]:
            P, _ = oracle.exact(p, oracle.phi_table_st(g, K=3, level=level), want_grad=False)
            assert abs(P - want) < 1e-13
    x = np.array([[2, 2, 1, 2, 2, 2]], dtype=np.uint8)
    assert oracle.phi_st(series, x[0], level=1) == 1
    assert oracle.phi_st(series, x[0], level=2) == 0
    Y, _ = oracle.eval_unknown(series, x, None, which=1, level=2)
    assert Y.tolist() == [0]


def test_exact_partials_against_closed_form_derivatives():
    """The brute-force partial G*[i][1] - G*[i][0] is dP/dp_i; compare with a
    central difference of the bridge's closed form and the series product."""
    pb = np.array([0.6, 0.7, 0.8, 0.55, 0.9])
    _, Gx = oracle.exact(oracle.state_probs_binary(pb), oracle.phi_table_st(_bridge()))
    for i in range(5):
        d = 1e-6
        hi, lo = pb.copy(), pb.copy()
        hi[i] += d
        lo[i] -= d
        fd = (_bridge_closed_form(hi) - _bridge_closed_form(lo)) / (2 * d)
        assert abs((Gx[i, 1] - Gx[i, 0]) - fd) < 1e-8
    ps = np.array([0.9, 0.8, 0.7, 0.95])
    series = _graph(5, [(i, i + 1) for i in range(4)], 0, 4)
    _, Gs = oracle.exact(oracle.state_probs_binary(ps), oracle.phi_table_st(series))
    for i in range(4):
        assert abs(Gs[i, 1] - np.prod(np.delete(ps, i))) < 1e-14
        assert Gs[i, 0] == 0.0


def test_tiny_reference_sets_from_two_routes():
    """Section 2.2 (binary case): the lower / upper reference sets of s-t
    connectivity are the minimal cut / path sets.  Brute force over all 2^20
    states (oracle) and graph enumeration (input generators) must agree."""
    c = WL.configs.tiny(N=10)
    table = oracle.phi_table_st(c["graph"])
    lo, up = oracle.reference_sets(table, c["n"], 2)
    assert set(map(bytes, lo)) == set(map(bytes, c["lower"]))
    assert set(map(bytes, up)) == set(map(bytes, c["upper"]))


def test_complete_refs_classify_every_state():
    """With complete reference sets every one of the 2^20 states is classified,
    exactly as the Phi table says, and never on both sides."""
    c = WL.configs.tiny(N=10)
    n = c["n"]
    table = oracle.phi_table_st(c["graph"])
    idx = np.arange(1 << n, dtype=np.uint64)
    states = ((idx[:, None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8)
    flags, _, _ = oracle.classify(c["lower"], c["upper"], states, mode=1)
    assert np.all((flags == 1) == (table == 0))
    assert np.all((flags == 2) == (table == 1))


def test_tiny_estimate_within_3_se_of_exact():
    c = WL.configs.tiny(N=200_000)
    table = oracle.phi_table_st(c["graph"])
    P, Gx = oracle.exact(c["p"], table)
    lower, upper = c["lower"][:-3], c["upper"][:-15]
    x = oracle.sample(c["p"], c["seed"], 0, 0, c["N"])
    fl, _, _ = oracle.classify(lower, upper, x, mode=0)
    Y, _ = oracle.eval_unknown(c["graph"], x, fl)
    est = oracle.estimate(oracle.counts(fl, Y))
    assert abs(est[3] - P) <= 3 * est[4]
    # Score-function partials within 3 standard errors of the exact ones.
    cnt, G = oracle.grad(c["p"], x, Y)
    N = c["N"]
    for i in range(c["n"]):
        for s in range(2):
            pi = c["p"][i, s]
            mean = cnt[i, s] / N
            se = math.sqrt(mean * (1 - mean) / N) / pi
            assert abs(G[i, s] - Gx[i, s]) <= 3 * se + 1e-12


# ------------------------------------------------------------- invariants ----

def test_rsr_equals_plain_monte_carlo_and_invariants():
    """I1: upper-flagged samples have Phi = 1 and lower-flagged ones Phi = 0;
    I2: no sample on both sides; I4: the RSR estimate equals plain Monte Carlo
    on the same samples; I5: p_U <= P <= 1 - p_L."""
    c = WL.configs.graph2(N=20_000)
    lower, upper = c["lower"][:3000], c["upper"][:3000]
    x = oracle.sample(c["p"], c["seed"], 0, 0, c["N"])
    fc, _, _ = oracle.classify(lower, upper, x, mode=1)
    Yall, _ = oracle.eval_unknown(c["graph"], x, None, which=1)
    assert np.all(Yall[(fc & 2) > 0] == 1)
    assert np.all(Yall[(fc & 1) > 0] == 0)
    assert not np.any(fc == 3)
    fl, _, _ = oracle.classify(lower, upper, x, mode=0)
    Y, nev = oracle.eval_unknown(c["graph"], x, fl)
    np.testing.assert_array_equal(Y, Yall)
    est = oracle.estimate(oracle.counts(fl, Y))
    assert est[3] == Yall.mean()
    assert est[1] <= est[3] <= 1 - est[0]
    assert nev == int((fl == 0).sum())


def test_monotone_under_common_random_numbers():
    """I6: raising one survival probability under the same seed never lowers any
    state, so Y and P are non-decreasing."""
    c = WL.configs.graph2(N=5_000)
    p = c["p"][:, 1].copy()
    x0 = oracle.sample(c["p"], 7, 0, 0, c["N"])
    for i in (0, 100, 294):
        q = p.copy()
        q[i] = min(1.0, q[i] + 0.05)
        x1 = oracle.sample(oracle.state_probs_binary(q), 7, 0, 0, c["N"])
        assert np.all(x1 >= x0)
        Y0, _ = oracle.eval_unknown(c["graph"], x0, None, which=1)
        Y1, _ = oracle.eval_unknown(c["graph"], x1, None, which=1)
        assert np.all(Y1 >= Y0)


def test_multistate_levels_nested_and_exact():
    """I7: Y at level 2 <= Y at level 1 per sample.  On a 3-state bridge the
    brute-force P(S >= k) matches the Monte Carlo estimate within 3 SE."""
    g = _bridge()
    rng = np.random.default_rng(12)
    p = rng.dirichlet([1.0, 2.0, 4.0], size=5)
    x = oracle.sample(p, 3, 0, 0, 100_000)
    Ys = {}
    for level in (1, 2):
        table = oracle.phi_table_st(g, K=3, level=level)
        P, _ = oracle.exact(p, table, want_grad=False)
        Y, _ = oracle.eval_unknown(g, x, None, which=1, level=level)
        Ys[level] = Y
        se = math.sqrt(P * (1 - P) / x.shape[0])
        assert abs(Y.mean() - P) <= 3 * se
        lo, up = oracle.reference_sets(table, 5, 3)
        fl, _, _ = oracle.classify(lo, up, x, mode=0)
        assert np.all(fl != 0)
        np.testing.assert_array_equal(fl == 2, Y == 1)
    assert np.all(Ys[2] <= Ys[1])
