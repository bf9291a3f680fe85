"""The stage-cell interpreter on the GPU: random valid programs against the
literal interpreter, and the patterns re-expressed as cells against the
fixed kernels, bit for bit."""
import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W
from tests import programs as P
from tests.brute import brute_program

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cells(prog):
    return [A.cell(c["op"], c["node"], c["peer"], c["tlo"], c["tref"], c["thi"], c["skip"], bool(c["distinct"]),
                   c["agg"], c["threshold"]) for c in prog]


def _run(G, prog, delta, k):
    out = A.amlm_mine_program(G, _cells(prog), delta, k)
    A.amlm_graph_sync(G)
    return A.to_u32(out)


@pytest.mark.parametrize("seed", range(12))
def test_random_programs_equal_literal_interpreter(seed):
    rng = np.random.default_rng(9300 + seed)
    g = W.random_small(seed + 930, n_edges=int(rng.integers(1, 150)), n_vertices=int(rng.integers(2, 12)),
                       t_range=int(rng.integers(1, 40)))
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    for _ in range(12):
        prog = P.random_program(rng)
        delta, k = int(rng.integers(0, 30)), int(rng.integers(1, 4))
        got = _run(G, prog, delta, k)
        ref = brute_program(g.src, g.dst, g.ts, prog, delta, k)
        np.testing.assert_array_equal(got.astype(np.uint64), ref, err_msg=str(prog))
    G.close()


def test_patterns_as_programs_equal_fixed_kernels():
    g = W.mid(217, scale=0.02)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    for k in (2, 3):
        fixed = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_FAN_OUT | A.AMLM_FAN_IN | A.AMLM_SG | A.AMLM_DEG_OUT |
                                                 A.AMLM_DEG_IN, 86400, 2, k)))
        unord = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_SG | A.AMLM_SG_UNORDERED, 86400, 2, k)))
        A.amlm_graph_sync(G)
        for prog, ref in ((P.FAN_OUT, fixed[0]), (P.FAN_IN, fixed[1]), (P.SG, fixed[2]), (P.DEG_OUT, fixed[3]),
                          (P.DEG_IN, fixed[4]), (P.SG_UNORDERED, unord[0])):
            np.testing.assert_array_equal(_run(G, prog, 86400, k), ref)
    # anchored cycles: every cycle once, from its last edge
    first = oracle.count_cycles_first(g.src, g.dst, g.ts, g.n_vertices, 86400, 5)
    for l in (2, 3, 4, 5):
        assert int(_run(G, P.cycle_anchored(l), 86400, 1).astype(np.uint64).sum()) == int(first[l])
    G.close()


def test_invalid_programs_are_rejected():
    g = W.random_small(1, n_edges=30, n_vertices=5, t_range=10)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    bad = [
        [P.C(P.FOR_OUT, 2)],                                     # vertex 2 not bound yet
        [P.C(P.PROBE, P.U, peer=P.V), P.C(P.FOR_OUT, P.U)],      # probe not last
        [P.C(P.FOR_OUT, P.U, tlo=P.AFTER, tref=0)],              # time reference not earlier
        [P.C(P.FOR_OUT, P.U, skip=(2,))],                        # skips an unbound vertex
        [P.C(7, P.U)],                                           # unknown operation
        [P.C(P.FOR_OUT, P.U)] * 7,                               # too many cells
    ]
    for prog in bad:
        with pytest.raises(A.AmlmError) as ei:
            _run(G, prog, 10, 1)
        assert ei.value.status == 1
    G.close()
