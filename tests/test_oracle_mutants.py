"""Mutation check of the oracle's pins (CPU only).

Each mutant is a copy of oracle/oracle.c with one plausible mistake planted
(a swapped constant, an off-by-one, a flipped comparison, a dropped term, a
wrong index).  It is compiled to a temporary library and the pin suites
(test_oracle_pins.py, test_oracle_boundary.py, test_oracle_global.py,
test_oracle_flow.py) run against it in a subprocess; every mutant must make
at least one pin fail.  This shows that the pins constrain every part of the
oracle, not only that the oracle passes them."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "philox multipliers swapped": ("const uint32_t mulA = 0xD2511F53u, mulB = 0xCD9E8D57u;",
                                   "const uint32_t mulA = 0xCD9E8D57u, mulB = 0xD2511F53u;"),
    "philox second key not bumped": ("k1 += weyl1;", "k1 += 0u;"),
    "philox output words permuted": ("out[0] = c0; out[1] = c1;", "out[0] = c1; out[1] = c0;"),
    "counter: component group i/4": ("uint32_t hi_ctr[4] = {(uint32_t)(i >> 3),",
                                      "uint32_t hi_ctr[4] = {(uint32_t)(i >> 2),"),
    "draw: wrong half of the block": ("const int j = i & 7;", "const int j = (i + 1) & 7;"),
    "draw: low half from the high block": ("{(uint32_t)(i >> 3) | 0x80000000u,",
                                           "{(uint32_t)(i >> 3),"),
    "draw: halves swapped": ("return (block_half(hi, j) << 16) | block_half(lo, j);",
                             "return (block_half(lo, j) << 16) | block_half(hi, j);"),
    "threshold: cumulative off by one state": ("acc = acc + p[(size_t)i * K + (s - 1)];",
                                               "acc = acc + p[(size_t)i * K + s];"),
    "state: strict threshold comparison": ("if (u >= C[(size_t)i * (K - 1) + (s - 1)]) state += 1;",
                                           "if (u > C[(size_t)i * (K - 1) + (s - 1)]) state += 1;"),
    "lower test: >= instead of >": ("if (x[i] > r[i]) return 0;", "if (x[i] >= r[i]) return 0;"),
    "upper test: <= instead of <": ("if (x[i] < r[i]) return 0;", "if (x[i] <= r[i]) return 0;"),
    "no lower precedence": ("if (mode == 1 || cl == 0) {", "if (1) {"),
    "Phi ignores the level": ("if ((int)x[e] < level) continue;", "if ((int)x[e] < 1) continue;"),
    "Phi (global): lower-flagged samples get Y = 1": ("if (which == 0 && (flags[h] & 1)) {\n            Y[h] = 0;",
                                                      "if (which == 0 && (flags[h] & 1)) {\n            Y[h] = 1;"),
    "Phi (s-t): lower-flagged samples get Y = 1": (
        "schedule(dynamic, 256) reduction(+ : evaluated)\n    for (int64_t h = 0; h < N; ++h) {\n"
        "        const uint8_t* xh = x + (size_t)h * n_edges;\n        if (which == 0 && (flags[h] & 1)) {\n"
        "            Y[h] = 0;",
        "schedule(dynamic, 256) reduction(+ : evaluated)\n    for (int64_t h = 0; h < N; ++h) {\n"
        "        const uint8_t* xh = x + (size_t)h * n_edges;\n        if (which == 0 && (flags[h] & 1)) {\n"
        "            Y[h] = 1;"),
    "estimate drops evaluated unknowns": ("double P = (double)(counts[1] + counts[4]) / Nd;",
                                          "double P = (double)(counts[1]) / Nd;"),
    "coefficient of variation inverted": ("sqrt((1.0 - P) / (Nd * P))", "sqrt(P / (Nd * (1.0 - P)))"),
    "gradient counts the wrong state": ("counts[(size_t)i * K + xh[i]] += 1;",
                                        "counts[(size_t)i * K + (K - 1 - xh[i])] += 1;"),
    "gradient divides by the wrong probability": (
        "(double)counts[(size_t)i * K + s] / ((double)N * pv)",
        "(double)counts[(size_t)i * K + s] / ((double)N * p[(size_t)i * K])"),
    "brute force: state probability uses state 0": ("for (int i = 0; i < n; ++i) prob *= p[(size_t)i * K + x[i]];\n        P += prob;",
                                                     "for (int i = 0; i < n; ++i) prob *= p[(size_t)i * K];\n        P += prob;"),
    "paper encoding: down-set strict": ("(m <= (int)r[i] ? 1 : 0)", "(m < (int)r[i] ? 1 : 0)"),
    "counts: both-flag samples counted upper": ("if (lo) nL += 1;\n        else if (up) nU += 1;",
                                               "if (lo && !up) nL += 1;\n        else if (up) nU += 1;"),
    "boundary: crossing raise kept": ("x[i] -= 1;\n                    break;", "break;"),
    "boundary: crossing lowering kept": ("x[i] += 1;\n                    break;", "break;"),
    "boundary: components visited in reverse": ("for (int i = 0; i < n; ++i) {\n        if (!start) {",
                                                "for (int i = n - 1; i >= 0; --i) {\n        if (!start) {"),
    "boundary: sides swapped": ("        if (!start) {\n            while", "        if (start) {\n            while"),
    "global: the left-out edge is still used": ("if (e == skip || x[e] < 1) continue;",
                                                "if (x[e] < 1) continue;"),
    "global: bridges ignored for level 2": ("if (reach_count(n_nodes, n_edges, eu, ev, x, e) < n_nodes) return 1;",
                                            "if (reach_count(n_nodes, n_edges, eu, ev, x, e) < 0) return 1;"),
    "global: strict level test": ("return or_state_global(n_nodes, n_edges, eu, ev, x) >= level;",
                                  "return or_state_global(n_nodes, n_edges, eu, ev, x) > level;"),
    "global: node 0 not counted": ("    seen[0] = 1;\n    queue[tail++] = 0;",
                                   "    seen[0] = 1;\n    queue[tail++] = 0;\n    tail += 0 * head++;"),
    "flow: reverse capacity ignores the flow": ("else if (ev[e] == u) { w = eu[e]; spare = x[e] + flow[e]; }",
                                                "else if (ev[e] == u) { w = eu[e]; spare = x[e]; }"),
    "flow: push sign flipped": ("if (from == eu[e]) flow[e] += push; else flow[e] -= push;",
                                "if (from == eu[e]) flow[e] -= push; else flow[e] += push;"),
    "flow: one augmenting path only": ("        total += push;\n    }", "        total += push;\n        break;\n    }"),
}
PIN_FILES = ["test_oracle_pins.py", "test_oracle_boundary.py", "test_oracle_global.py",
             "test_oracle_flow.py", "test_oracle_properties.py"]


def _run(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    path_c = os.path.join(tmp, f"m{abs(hash(name))}.c")
    path_so = path_c[:-2] + ".so"
    open(path_c, "w").write(src.replace(old, new, 1) if old else src)
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", path_so, path_c, "-lm"], check=True, capture_output=True)
    env = dict(os.environ, RSR_ORACLE_LIB=path_so, OMP_NUM_THREADS="2")
    # A mutant can also loop forever (a flow that never saturates): a pin that
    # times out has caught it too.
    try:
        r = subprocess.run([sys.executable, "-m", "pytest",
                            *[os.path.join(ROOT, "tests", f) for f in PIN_FILES],
                            "-x", "-q", "-p", "no:cacheprovider", "--timeout", "20"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    except subprocess.TimeoutExpired:
        return name, "timeout"
    return name, r.returncode


def test_every_mutant_is_killed():
    """pytest exits with 1 when a test failed (a pin caught the mutant); any
    other non-zero code (collection or usage error, internal error, no tests)
    is not a catch.  The unmodified source goes through the same build and run
    first and must pass."""
    with tempfile.TemporaryDirectory() as tmp:
        _, rc0 = _run("unmutated", "", "", tmp)
        assert rc0 == 0, f"the unmutated oracle fails its pins in the harness (rc {rc0})"
        with cf.ThreadPoolExecutor(max_workers=6) as ex:
            results = list(ex.map(lambda kv: _run(kv[0], kv[1][0], kv[1][1], tmp), MUTANTS.items()))
    caught = {name for name, rc in results if rc == 1 or rc == "timeout"}
    odd = {name: rc for name, rc in results if name not in caught and rc != 0}
    survivors = [name for name, rc in results if rc == 0]
    assert not odd, f"mutant runs that ended neither passing nor failing: {odd}"
    assert not survivors, f"mutants not caught by any pin: {survivors}"
