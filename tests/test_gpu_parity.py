"""GPU parity: every output of the HIP path against the plain CPU oracle on the
same seeded inputs.  Integer outputs (samples, flags, match counts, Y, counts,
estimates) must be bit-exact; the fp32 gradient must be within 1e-5 relative
of the fp64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL
from helpers import pad_bits, unpack_states

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-5


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _sample(ctx, p, seed, stream, first, N):
    m = R.Model(ctx, p)
    xs = R.rsr_sample(ctx, m, seed, stream, first, N)
    return m, xs


# ---------------------------------------------------------------- sampler ----

@pytest.mark.parametrize("n,K,N,first,stream", [
    (20, 2, 1000, 0, 0),
    (295, 2, 4099, 12345, 7),
    (37, 5, 777, (1 << 32) - 300, 3),
    (64, 3, 513, 0, 0),
    (1, 2, 65, 5, 0),
    (1250, 2, 300, 99, 1),
])
def test_sample_bit_identical(rsr_ctx, n, K, N, first, stream):
    rng = np.random.default_rng(n * 100 + K)
    p = rng.dirichlet(np.ones(K), size=n)
    p[0] = 0.0
    p[0, K - 1] = 1.0          # a component that is always in the top state
    if n > 1:
        p[1] = 0.0
        p[1, 0] = 1.0          # and one that is always in state 0
    seed = 0x123456789ABCDEF ^ n
    m, xs = _sample(rsr_ctx, p, seed, stream, first, N)
    words = _np(xs)
    assert words.shape == (m.words, N)
    assert pad_bits(words, n, K) == 0
    got = unpack_states(words, n, K)
    want = oracle.sample(p, seed, stream, first, N)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("kind,n,K,N", [("dirichlet", 64, 16, 200_000), ("uniform", 40, 16, 50_000),
                                         ("dyadic", 33, 2, 70_001)])
def test_sample_ties_of_the_high_half(rsr_ctx, kind, n, K, N):
    """The sampler decides u >= C from the high 16 bits of u unless they equal
    C's high half (the second Philox block then decides).  With 64 x 15
    thresholds per sample, 2e5 samples hit that case a few thousand times;
    uniform K = 16 thresholds (s * 2^28) and dyadic ones (multiples of 2^16)
    have zero low halves, where the equal high half alone means u >= C."""
    rng = np.random.default_rng(n + K)
    if kind == "dirichlet":
        p = rng.dirichlet(np.ones(K), size=n)
    elif kind == "uniform":
        p = np.full((n, K), 1.0 / K)
    else:
        q = rng.integers(1, 65536, n) / 65536.0
        p = np.stack([q, 1.0 - q], axis=1)
    m, xs = _sample(rsr_ctx, p, 0xC0FFEE, 3, 17, N)
    got = unpack_states(_np(xs), n, K)
    want = oracle.sample(p, 0xC0FFEE, 3, 17, N)
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------------- classifier ----

FORMS = (R.RSR_POPCOUNT, R.RSR_MFMA, R.RSR_MFMA_FP4, R.RSR_AUTO)


def _classify_both(ctx, cfg, N, lower, upper, level=1):
    """Every kernel form (and the automatic choice, whose LABEL mode on
    consistent rows is the cascade with FP4 split rounds) in both modes, and
    the persistent cascade in LABEL mode on consistent rows; returns
    {form: (label flags, count flags or None, match counts or None)} and the
    oracle's answers."""
    n, K = cfg["n"], cfg["K"]
    p = cfg["p"]
    m, xs = _sample(ctx, p, cfg["seed"], cfg["stream"], 0, N)
    refs = R.Refs(ctx, n, K, lower, upper)
    got = {}
    for form in FORMS:
        fl = R.rsr_classify(ctx, refs, xs, N, R.RSR_LABEL, form)
        fc, mt = R.rsr_classify(ctx, refs, xs, N, R.RSR_COUNT, form, want_match=True)
        got[form] = (_np(fl), _np(fc), _np(mt).view(np.uint32))
    if refs.consistent and n * (K - 1) <= 1280:
        got[R.RSR_PERSIST] = (_np(R.rsr_classify(ctx, refs, xs, N, R.RSR_LABEL, R.RSR_PERSIST)),
                              None, None)
    x = oracle.sample(p, cfg["seed"], cfg["stream"], 0, N)
    ol, _, _ = oracle.classify(lower, upper, x, mode=0)
    oc, mL, mU = oracle.classify(lower, upper, x, mode=1)
    return got, (ol, oc, mL, mU), (m, xs, refs, x)


def _assert_classify(got, want):
    ol, oc, mL, mU = want
    for form, (fl, fc, mt) in got.items():
        np.testing.assert_array_equal(fl, ol, err_msg=f"label flags, form {form}")
        if fc is None:
            continue
        np.testing.assert_array_equal(fc, oc, err_msg=f"count flags, form {form}")
        np.testing.assert_array_equal(mt[:, 0], mL, err_msg=f"lower matches, form {form}")
        np.testing.assert_array_equal(mt[:, 1], mU, err_msg=f"upper matches, form {form}")


def test_refs_consistency_flag(rsr_ctx):
    cfg = WL.configs.tiny(N=10)
    assert R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"]).consistent
    sc = WL.configs.scaling(N=10, R_U=200, R_L=200)
    assert not R.Refs(rsr_ctx, sc["n"], 2, sc["lower"], sc["upper"]).consistent
    n = 5
    lower = np.array([[1, 1, 0, 1, 1]], dtype=np.uint8)
    upper = np.array([[0, 1, 0, 0, 0], [0, 0, 1, 0, 0]], dtype=np.uint8)
    assert not R.Refs(rsr_ctx, n, 2, lower, upper).consistent     # (0,1,0,0,0) <= lower row
    assert R.Refs(rsr_ctx, n, 2, lower, upper[1:]).consistent
    assert R.Refs(rsr_ctx, n, 2, lower[:0], upper).consistent


@pytest.mark.parametrize("name", ["graph2", "multi"])
def test_refs_consistency_large_sets(rsr_ctx, name):
    """The consistency check over thousands of rows per side (in the FP4 form
    when the handle has matrix-core operands): the structural sets are
    consistent, one upper row appended anywhere below a lower row (equal to
    the last lower row, or a lower row with working components removed) makes
    them inconsistent, and an all-working upper row keeps them consistent."""
    if name == "graph2":
        cfg = WL.configs.graph2(N=1)
        n, K = cfg["n"], 2
        lower, upper = cfg["lower"][:3000], cfg["upper"][:2500]
    else:
        cfg = WL.configs.multi(N=1, R_per_level=4000)
        n, K = cfg["n"], 3
        lower, upper = cfg["levels"][2]["lower"], cfg["levels"][2]["upper"]
    assert R.Refs(rsr_ctx, n, K, lower, upper).consistent
    rng = np.random.default_rng(3)
    below = lower[len(lower) // 2].copy()
    on = np.nonzero(below)[0]
    below[rng.choice(on, size=len(on) // 3, replace=False)] = 0
    for extra in (lower[-1:], below[None, :]):
        bad = np.concatenate([upper, extra])
        assert not R.Refs(rsr_ctx, n, K, lower, bad).consistent
        assert not R.Refs(rsr_ctx, n, K, lower, bad[::-1]).consistent
    top = np.full((1, n), K - 1, np.uint8)
    assert R.Refs(rsr_ctx, n, K, lower, np.concatenate([upper, top])).consistent


def test_classify_tiny_complete_refs(rsr_ctx):
    cfg = WL.configs.tiny(N=100_000)
    got, want, _ = _classify_both(rsr_ctx, cfg, cfg["N"], cfg["lower"], cfg["upper"])
    _assert_classify(got, want)
    # complete reference sets leave nothing unclassified
    assert int((got[R.RSR_POPCOUNT][0] & 3 == 0).sum()) == 0


def test_classify_graph2_subset(rsr_ctx):
    cfg = WL.configs.graph2(N=30_011)
    lower, upper = cfg["lower"][:3000], cfg["upper"][:2500]
    got, want, _ = _classify_both(rsr_ctx, cfg, cfg["N"], lower, upper)
    _assert_classify(got, want)


def test_classify_bernoulli_rows_both_sides(rsr_ctx):
    cfg = WL.configs.scaling(N=20_000, R_U=1500, R_L=1700)
    got, want, _ = _classify_both(rsr_ctx, cfg, cfg["N"], cfg["lower"], cfg["upper"])
    _assert_classify(got, want)


def test_classify_bernoulli_dense_matches(rsr_ctx):
    # Denser lower rows make lower matches common, so both-flag samples and the
    # lower precedence of the LABEL mode are exercised.
    n = 40
    rng = np.random.default_rng(5)
    p = WL.configs.binary_model(rng.uniform(0.2, 0.6, n))
    cfg = {"n": n, "K": 2, "p": p, "seed": 77, "stream": 2}
    lower = WL.bernoulli_rows(500, n, 0.8, seed=6)
    upper = WL.bernoulli_rows(400, n, 0.15, seed=7)
    got, want, _ = _classify_both(rsr_ctx, cfg, 9_999, lower, upper)
    _assert_classify(got, want)
    assert int((want[1] == 3).sum()) > 0


@pytest.mark.parametrize("level", [1, 2])
def test_classify_multistate_levels(rsr_ctx, level):
    cfg = WL.configs.multi(N=10_007, R_per_level=4000)
    lv = cfg["levels"][level]
    got, want, _ = _classify_both(rsr_ctx, cfg, cfg["N"], lv["lower"], lv["upper"])
    _assert_classify(got, want)


@pytest.mark.parametrize("RL,RU,N", [(0, 50, 1000), (60, 0, 1000), (0, 0, 100), (33, 31, 1),
                                     (70, 65, 63), (70, 65, 65)])
def test_classify_edge_shapes(rsr_ctx, RL, RU, N):
    n, K = 70, 3
    rng = np.random.default_rng(RL * 7 + RU + N)
    p = rng.dirichlet([1.0, 1.0, 3.0], size=n)
    cfg = {"n": n, "K": K, "p": p, "seed": 9, "stream": 0}
    lower = rng.integers(1, 3, size=(RL, n)).astype(np.uint8)
    upper = (rng.random((RU, n)) < 0.1).astype(np.uint8)
    if RL > 2:
        lower[1] = lower[0]     # duplicate rows are legal
    got, want, _ = _classify_both(rsr_ctx, cfg, N, lower, upper)
    _assert_classify(got, want)


# ---------------------------------------------------- eval / estimate / grad --

def _full_path(ctx, cfg, N, lower, upper, level=1, form=R.RSR_POPCOUNT):
    n, K = cfg["n"], cfg["K"]
    g = cfg["graph"]
    m = R.Model(ctx, cfg["p"])
    refs = R.Refs(ctx, n, K, lower, upper)
    sysm = R.System(ctx, g, K=K, level=level)
    est, buf = R.stage2(ctx, m, refs, sysm, N, cfg["seed"], stream_id=cfg["stream"], form=form)
    Gc = R.rsr_grad(ctx, m, buf.samples, buf.Y, N, want_counts=True)
    return est, buf, Gc, (m, refs, sysm)


def _oracle_path(cfg, N, lower, upper, level=1):
    x = oracle.sample(cfg["p"], cfg["seed"], cfg["stream"], 0, N)
    fl, _, _ = oracle.classify(lower, upper, x, mode=0)
    Y, nev = oracle.eval_unknown(cfg["graph"], x, fl, which=0, level=level)
    cnt = oracle.counts(fl, Y)
    est = oracle.estimate(cnt)
    c, G = oracle.grad(cfg["p"], x, Y)
    return x, fl, Y, nev, cnt, est, c, G


def _assert_estimate(est, cnt, oest):
    for k, name in enumerate(oracle.COUNT_NAMES):
        assert est[name] == int(cnt[k]), name
    for k, name in enumerate(oracle.EST_NAMES):
        assert est[name] == oest[k] or (np.isinf(est[name]) and np.isinf(oest[k])), name


def _assert_grad(G, counts, c, Gref):
    np.testing.assert_array_equal(counts.view(np.uint64), c)
    G = G.astype(np.float64)
    nz = Gref != 0
    rel = np.abs(G[nz] - Gref[nz]) / np.abs(Gref[nz])
    assert rel.max(initial=0.0) <= GRAD_RTOL
    assert np.all(G[~nz] == 0.0)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name", ["tiny", "graph2"])
def test_full_path_bit_exact(rsr_ctx, name, form):
    if name == "tiny":
        cfg = WL.configs.tiny(N=100_000)
        lower, upper = cfg["lower"][:-4], cfg["upper"][:-20]   # partial refs -> unknowns
    else:
        cfg = WL.configs.graph2(N=50_000)
        lower, upper = cfg["lower"][:2000], cfg["upper"][:2000]
    N = cfg["N"]
    est, buf, (G, counts), _ = _full_path(rsr_ctx, cfg, N, lower, upper, form=form)
    x, fl, Y, nev, cnt, oest, c, Gref = _oracle_path(cfg, N, lower, upper)
    np.testing.assert_array_equal(_np(buf.flags), fl)
    np.testing.assert_array_equal(_np(buf.Y), Y)
    assert int(_np(buf.n_eval)[0]) == nev
    assert nev > 0
    _assert_estimate(est, cnt, oest)
    _assert_grad(_np(G), _np(counts), c, Gref)


def test_eval_all_is_plain_mc(rsr_ctx):
    cfg = WL.configs.graph2(N=20_000)
    N = cfg["N"]
    m, xs = _sample(rsr_ctx, cfg["p"], cfg["seed"], 0, 0, N)
    sysm = R.System(rsr_ctx, cfg["graph"])
    nev = torch.zeros(1, dtype=torch.int64, device="cuda")
    Y = R.rsr_eval_unknown(rsr_ctx, sysm, xs, N, None, which=R.RSR_ALL, n_evaluated=nev)
    x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, N)
    Yo, _ = oracle.eval_unknown(cfg["graph"], x, None, which=1)
    np.testing.assert_array_equal(_np(Y), Yo)
    assert int(_np(nev)[0]) == N


def test_multistate_full_path(rsr_ctx):
    cfg = WL.configs.multi(N=20_000, R_per_level=4000)
    N = cfg["N"]
    for level in (1, 2):
        lv = cfg["levels"][level]
        est, buf, (G, counts), _ = _full_path(rsr_ctx, cfg, N, lv["lower"], lv["upper"], level)
        x, fl, Y, nev, cnt, oest, c, Gref = _oracle_path(cfg, N, lv["lower"], lv["upper"], level)
        np.testing.assert_array_equal(_np(buf.flags), fl)
        np.testing.assert_array_equal(_np(buf.Y), Y)
        _assert_estimate(est, cnt, oest)
        _assert_grad(_np(G), _np(counts), c, Gref)


def test_estimate_bounds_only(rsr_ctx):
    cfg = WL.configs.tiny(N=5000)
    m, xs = _sample(rsr_ctx, cfg["p"], cfg["seed"], 0, 0, cfg["N"])
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"][:5], cfg["upper"][:5])
    fl = R.rsr_classify(rsr_ctx, refs, xs, cfg["N"])
    est = R.rsr_estimate(rsr_ctx, fl, None, cfg["N"])
    cnt = oracle.counts(_np(fl))
    oest = oracle.estimate(cnt, has_Y=False)
    assert est["n_u_up"] == 0
    assert np.isnan(est["P"]) and np.isnan(oest[3])
    assert est["p_L"] == oest[0] and est["p_U"] == oest[1] and est["p_u"] == oest[2]


# ------------------------------------------------ full-size sampled checks ----

@pytest.mark.parametrize("form", FORMS)
def test_graph2_full_size_sampled(rsr_ctx, form):
    """The benchmark configuration (119 nodes / 295 edges, 1e4 + 1e4 rows,
    N = 1e6), checked on 3000 sampled indices one by one."""
    cfg = WL.configs.graph2()
    N = cfg["N"]
    m = R.Model(rsr_ctx, cfg["p"])
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"])
    sysm = R.System(rsr_ctx, cfg["graph"])
    est, buf = R.stage2(rsr_ctx, m, refs, sysm, N, cfg["seed"], form=form)
    G, counts = R.rsr_grad(rsr_ctx, m, buf.samples, buf.Y, N, want_counts=True)
    rng = np.random.default_rng(123)
    idx = np.unique(np.concatenate([rng.integers(0, N, 3000), [0, N - 1]])).astype(np.uint64)
    x = oracle.sample_at(cfg["p"], cfg["seed"], 0, idx)
    got_x = unpack_states(_np(buf.samples)[:, idx.astype(np.int64)], cfg["n"], 2)
    np.testing.assert_array_equal(got_x, x)
    fl, _, _ = oracle.classify(cfg["lower"], cfg["upper"], x, mode=0)
    np.testing.assert_array_equal(_np(buf.flags)[idx.astype(np.int64)], fl)
    Y, _ = oracle.eval_unknown(cfg["graph"], x, fl, which=0)
    np.testing.assert_array_equal(_np(buf.Y)[idx.astype(np.int64)], Y)
    # Properties that hold at any size.
    assert est["N"] == N
    assert est["n_L"] + est["n_U"] + est["n_u"] == N
    assert est["n_both"] == 0
    assert est["p_U"] <= est["P"] <= 1.0 - est["p_L"]
    c = _np(counts).view(np.uint64)
    n_y1 = est["n_U"] + est["n_u_up"]
    assert np.all(c.sum(axis=1) == n_y1)
    G = _np(G).astype(np.float64)
    Gexp = c / (N * cfg["p"])
    nz = c > 0          # a bridge edge in state 0 never has Y = 1
    assert np.max(np.abs(G[nz] - Gexp[nz]) / Gexp[nz]) <= GRAD_RTOL
    assert np.all(G[~nz] == 0.0)


@pytest.mark.parametrize("form", FORMS)
def test_scaling_full_size_sampled_counts(rsr_ctx, form):
    """Kernel-only scaling workload (n = 295, 1e5 + 1e5 rows, N = 1e6) in
    COUNT mode, exact match counts on 300 sampled samples."""
    cfg = WL.configs.scaling()
    N = cfg["N"]
    m, xs = _sample(rsr_ctx, cfg["p"], cfg["seed"], 0, 0, N)
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"])
    fc, mt = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_COUNT, form, want_match=True)
    fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, form)
    rng = np.random.default_rng(7)
    idx = np.unique(rng.integers(0, N, 300)).astype(np.uint64)
    x = oracle.sample_at(cfg["p"], cfg["seed"], 0, idx)
    oc, mL, mU = oracle.classify(cfg["lower"], cfg["upper"], x, mode=1)
    ol, _, _ = oracle.classify(cfg["lower"], cfg["upper"], x, mode=0)
    ii = idx.astype(np.int64)
    mt = _np(mt).view(np.uint32)
    np.testing.assert_array_equal(_np(fc)[ii], oc)
    np.testing.assert_array_equal(mt[ii, 0], mL)
    np.testing.assert_array_equal(mt[ii, 1], mU)
    np.testing.assert_array_equal(_np(fl)[ii], ol)


def test_classify_forms_agree_and_deterministic(rsr_ctx):
    cfg = WL.configs.graph2(N=100_000)
    m, xs = _sample(rsr_ctx, cfg["p"], cfg["seed"], 0, 0, cfg["N"])
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"])
    runs = [_np(R.rsr_classify(rsr_ctx, refs, xs, cfg["N"], R.RSR_COUNT, f, want_match=True)[1])
            for f in (R.RSR_POPCOUNT, R.RSR_MFMA, R.RSR_MFMA_FP4, R.RSR_MFMA,
                      R.RSR_MFMA_FP4, R.RSR_POPCOUNT)]
    for r in runs[1:]:
        np.testing.assert_array_equal(r, runs[0])


def test_cascade_fp4_split_rounds_large_rows(rsr_ctx):
    """The 1250-edge graph (40 words per row) with 1e4 path / cut rows: the
    automatic LABEL cascade runs its split rounds in the FP4 form; labels equal
    the popcount cascade's and the oracle's."""
    sd = WL.configs.batched(n_scen=1, N=1, graphs=[7], ref_scale=0.05)
    sys_ = sd["systems"][0]
    n = sys_["n"]
    p = sd["jobs"][0]["p"]
    N = 3000
    m, xs = _sample(rsr_ctx, p, 3, 0, 0, N)
    refs = R.Refs(rsr_ctx, n, 2, sys_["lower"], sys_["upper"])
    assert refs.consistent
    auto = _np(R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_AUTO))
    pop = _np(R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_POPCOUNT))
    x = oracle.sample(p, 3, 0, 0, N)
    want, _, _ = oracle.classify(sys_["lower"], sys_["upper"], x, mode=0)
    print("rows", refs.R_L, refs.R_U, "unclassified", int((want == 0).sum()))
    np.testing.assert_array_equal(pop, want)
    np.testing.assert_array_equal(auto, want)


def test_persistent_cascade_long_rows(rsr_ctx):
    """2.2e4 path and cut rows of the 647-edge graph (21 words per row): the
    persistent cascade (round 0 on the vector ALU, the later rounds in one
    cooperative launch, compacted through per-block regions) and the
    automatic LABEL form (round kernels with growth 8 at this many rows).  A
    ragged N; labels equal the oracle's and the popcount cascade's, and a
    second call on the same buffers repeats them."""
    cfg = WL.configs.batched(n_scen=1, N=1, graphs=[5], ref_scale=1.0)
    sys_ = cfg["systems"][0]
    n = sys_["n"]
    p = cfg["jobs"][0]["p"]
    N = 6007
    m, xs = _sample(rsr_ctx, p, 5, 0, 0, N)
    refs = R.Refs(rsr_ctx, n, 2, sys_["lower"], sys_["upper"])
    assert refs.consistent and max(refs.R_L, refs.R_U) >= 16_384
    x = oracle.sample(p, 5, 0, 0, N)
    want, _, _ = oracle.classify(sys_["lower"], sys_["upper"], x, mode=0)
    for form in (R.RSR_PERSIST, R.RSR_AUTO):
        fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, form)
        first = _np(fl).copy()
        R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, form, flags=fl)
        np.testing.assert_array_equal(first, want, err_msg=f"form {form}")
        np.testing.assert_array_equal(_np(fl), want, err_msg=f"form {form}, second call")
    pop = _np(R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_POPCOUNT))
    np.testing.assert_array_equal(pop, want)


@pytest.mark.parametrize("form,per_cu", [(R.RSR_MFMA, 640), (R.RSR_MFMA, 512),
                                         (R.RSR_MFMA_FP4, 1024), (R.RSR_MFMA_FP4, 512)])
def test_classify_both_sample_tile_counts(rsr_ctx, form, per_cu):
    """graph2's width (295 bits) builds two sample-tile counts per matrix form
    (int8: 5 and 4, FP4: 8 and 4) and the launcher picks by N and the CU
    count; N = per_cu * CUs - 37 selects each of them once (a ragged last
    block).  Exact counts and labels on sampled indices and the tail."""
    cfg = WL.configs.graph2()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    N = per_cu * cus - 37
    m, xs = _sample(rsr_ctx, cfg["p"], cfg["seed"], 0, 0, N)
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"])
    fc, mt = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_COUNT, form, want_match=True)
    fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, form)
    rng = np.random.default_rng(per_cu)
    idx = np.unique(np.concatenate([rng.integers(0, N, 600), np.arange(N - 300, N)]))
    x = oracle.sample_at(cfg["p"], cfg["seed"], 0, idx.astype(np.uint64))
    oc, mL, mU = oracle.classify(cfg["lower"], cfg["upper"], x, mode=1)
    ol, _, _ = oracle.classify(cfg["lower"], cfg["upper"], x, mode=0)
    mt = _np(mt).view(np.uint32)
    np.testing.assert_array_equal(_np(fc)[idx], oc)
    np.testing.assert_array_equal(mt[idx, 0], mL)
    np.testing.assert_array_equal(mt[idx, 1], mU)
    np.testing.assert_array_equal(_np(fl)[idx], ol)


@pytest.mark.parametrize("n", [700, 1100, 1250])
def test_classify_wide_rows(rsr_ctx, n):
    """Wide rows (int8: 11, 18 and 20 K-steps, FP4: 6, 9 and 10) run with 3, 2
    and 2 (int8) and 4, 3 and 3 (FP4) sample tiles per wave; N = 3001 spans
    several blocks and a ragged tail.  Every form against the oracle."""
    rng = np.random.default_rng(n)
    p = WL.configs.binary_model(rng.uniform(0.85, 0.995, n))
    cfg = {"n": n, "K": 2, "p": p, "seed": 21, "stream": 1}
    # Rows built around some of the samples themselves (a sample's states
    # raised at random components, or cut down to a few of its surviving
    # ones), so that lower, upper, both and no matches all occur.
    x = oracle.sample(p, cfg["seed"], cfg["stream"], 0, 3001)
    lower = np.maximum(x[rng.integers(0, 3001, 300)], rng.random((300, n)) < 0.6).astype(np.uint8)
    upper = (x[rng.integers(0, 3001, 280)] & (rng.random((280, n)) < 0.1)).astype(np.uint8)
    got, want, _ = _classify_both(rsr_ctx, cfg, 3001, lower, upper)
    _assert_classify(got, want)
    assert all(int((want[1] == f).sum()) > 0 for f in (0, 1, 2, 3))


@pytest.mark.parametrize("n,K,N", [(40, 3, 3_000_001), (40, 3, 3_000_000), (33, 2, 17),
                                   (70, 4, 65_537), (70, 4, 65_536)])
def test_grad_counts_any_run_length(rsr_ctx, n, K, N):
    """The gradient kernel counts in bit-sliced chunks of at most 120 samples
    per thread; at N = 3e6 each thread walks about 180 samples, so the chunk
    boundary is crossed.  N a multiple of 4 takes four samples per load, other
    N one.  Counts against the oracle on the same samples and a seeded Y with
    about half ones; tiny and ragged N too."""
    rng = np.random.default_rng(n * K)
    p = rng.dirichlet(np.ones(K) * 2.0, size=n)
    m, xs = _sample(rsr_ctx, p, 99, 4, 0, N)
    Y = (rng.random(N) < 0.5).astype(np.uint8)
    G, counts = R.rsr_grad(rsr_ctx, m, xs, torch.from_numpy(Y).to(rsr_ctx.device), N,
                           want_counts=True)
    x = oracle.sample(p, 99, 4, 0, N)
    c, Gref = oracle.grad(p, x, Y)
    _assert_grad(_np(G), _np(counts), c, Gref)


@pytest.mark.parametrize("N,offset,with_Y", [(1_000_003, 0, True), (1_000_003, 1, True),
                                             (15, 0, True), (16, 0, False), (70_001, 3, False),
                                             (1_000_000, 0, False), (1 << 24, 0, True),
                                             ((1 << 24) + 37, 0, True)])
def test_estimate_counts_any_alignment(rsr_ctx, N, offset, with_Y):
    """Counts of rsr_estimate: 16-byte aligned flags and Y take the one-launch
    kernel (16 flags per load, a ragged tail of up to 15; a grid of at most
    1024 blocks, so from 2^24 flags on a thread takes more than four loads),
    others the
    per-byte kernels; flags hold every value 0..3 and Y is 0, 1 or larger
    (counted as 1).  Exact against the oracle, and repeated calls agree."""
    rng = np.random.default_rng(N + offset)
    fl = rng.integers(0, 4, N + offset).astype(np.uint8)
    Y = rng.choice(np.array([0, 1, 2, 255], dtype=np.uint8), N + offset)
    dev_f = torch.from_numpy(fl).to(rsr_ctx.device)[offset:]
    dev_Y = torch.from_numpy(Y).to(rsr_ctx.device)[offset:] if with_Y else None
    want = oracle.counts(fl[offset:], Y[offset:] if with_Y else None)
    oest = oracle.estimate(want, has_Y=with_Y)
    for _ in range(3):
        est = R.rsr_estimate(rsr_ctx, dev_f, dev_Y, N)
        for k, name in enumerate(oracle.COUNT_NAMES):
            assert est[name] == int(want[k]), name
        for k, name in enumerate(oracle.EST_NAMES[:3]):
            assert est[name] == oest[k], name


def test_estimate_after_long_queue(rsr_ctx):
    """rsr_estimate returns once the counting kernel's last block has
    published the call's sequence number next to the counts; with more than
    10 ms of work queued before it (two exhaustive classifications of 2^20
    samples against 5e4 + 5e4 rows) it synchronises the stream instead.  On
    consecutive calls with different flags, either way, the counts are those
    of the flags given, exact against the oracle."""
    cfg = WL.configs.scaling(N=1 << 20, R_U=50_000, R_L=50_000)
    N = cfg["N"]
    _, xs = _sample(rsr_ctx, cfg["p"], cfg["seed"], 0, 0, N)
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"])
    rng = np.random.default_rng(5)
    flag_sets = [rng.integers(0, 4, N).astype(np.uint8) for _ in range(4)]
    Y = rng.integers(0, 2, N).astype(np.uint8)
    dev_Y = torch.from_numpy(Y).to(rsr_ctx.device)
    dev = [torch.from_numpy(f).to(rsr_ctx.device) for f in flag_sets]
    torch.cuda.synchronize()
    for k, (f, d) in enumerate(zip(flag_sets, dev)):
        if k % 2 == 0:
            for _ in range(2):
                R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_COUNT, R.RSR_POPCOUNT)
        est = R.rsr_estimate(rsr_ctx, d, dev_Y, N)
        want = oracle.counts(f, Y)
        for j, name in enumerate(oracle.COUNT_NAMES):
            assert est[name] == int(want[j]), (k, name)


@pytest.mark.parametrize("g_idx,level", [(0, 1), (2, 1), (4, 1), (6, 1), (4, 2)])
def test_eval_all_graph_sizes(rsr_ctx, g_idx, level):
    """s-t evaluation on graphs of 50 to 360 nodes (one to several node words
    and edge rounds per lane), every sample evaluated, against the oracle;
    three-state edges for level 2."""
    g = WL.configs._batch_graph(g_idx)
    n = int(g["edge_u"].size)
    rng = np.random.default_rng(g_idx)
    K = level + 1
    p = rng.dirichlet(np.array([1.0, 4.0, 8.0][:K]), size=n) if K == 3 else \
        WL.configs.binary_model(rng.uniform(0.55, 0.95, n))
    N = 4099
    m, xs = _sample(rsr_ctx, p, 13, 2, 0, N)
    system = R.System(rsr_ctx, g, K=K, level=level)
    flags = torch.zeros(N, dtype=torch.uint8, device=rsr_ctx.device)
    Y = R.rsr_eval_unknown(rsr_ctx, system, xs, N, flags, which=R.RSR_ALL)
    x = oracle.sample(p, 13, 2, 0, N)
    want, _ = oracle.eval_unknown(g, x, np.zeros(N, dtype=np.uint8), which=1, level=level)
    got = _np(Y)
    np.testing.assert_array_equal(got, want)
    assert 0 < int(want.sum()) < N


@pytest.mark.parametrize("g", range(8))
def test_classify_forms_agree_every_width(rsr_ctx, g):
    """The eight batched graphs (120 to 1250 edges: 4 to 40 packed words, 2 to
    20 FP4 k-steps of 64) with 5 % of their reference rows: every form gives
    the popcount form's COUNT flags and match counts and its LABEL flags (the
    persistent cascade its LABEL flags), on a ragged N; the oracle checks
    sampled indices."""
    cfg = WL.configs.batched(n_scen=1, N=1, graphs=[g], ref_scale=0.05)
    sd = cfg["systems"][0]
    n, p = sd["n"], cfg["jobs"][0]["p"]
    N = 5003
    m, xs = _sample(rsr_ctx, p, 11, 0, 0, N)
    refs = R.Refs(rsr_ctx, n, 2, sd["lower"], sd["upper"])
    fc0, mt0 = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_COUNT, R.RSR_POPCOUNT, want_match=True)
    fc0, mt0 = _np(fc0).copy(), _np(mt0).view(np.uint32).copy()
    fl0 = _np(R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_POPCOUNT)).copy()
    for form in (R.RSR_MFMA, R.RSR_MFMA_FP4, R.RSR_AUTO):
        fc, mt = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_COUNT, form, want_match=True)
        np.testing.assert_array_equal(_np(fc), fc0, err_msg=f"COUNT flags, form {form}")
        np.testing.assert_array_equal(_np(mt).view(np.uint32), mt0, err_msg=f"counts, form {form}")
        fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, form)
        np.testing.assert_array_equal(_np(fl), fl0, err_msg=f"LABEL flags, form {form}")
    assert refs.consistent
    fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_PERSIST)
    np.testing.assert_array_equal(_np(fl), fl0, err_msg="LABEL flags, persistent cascade")
    idx = np.unique(np.concatenate([np.arange(0, N, 97), [N - 1]]))
    x = oracle.sample_at(p, 11, 0, idx.astype(np.uint64))
    oc, mL, mU = oracle.classify(sd["lower"], sd["upper"], x, mode=1)
    np.testing.assert_array_equal(fc0[idx], oc)
    np.testing.assert_array_equal(mt0[idx, 0], mL)
    np.testing.assert_array_equal(mt0[idx, 1], mU)
