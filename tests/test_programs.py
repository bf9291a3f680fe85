"""The stage-cell program semantics (literal CPU interpreter) against the
oracle: the paper's patterns re-expressed as cells give the oracle's
columns, and anchored cycle programs add up to the cycle count."""
import numpy as np
import pytest

import oracle
from paper_2604_12241_amd import workloads as W
from tests import programs as P
from tests.brute import brute_program


@pytest.mark.parametrize("seed", range(8))
def test_patterns_as_programs_equal_oracle(seed):
    rng = np.random.default_rng(9100 + seed)
    g = W.random_small(seed + 910, n_edges=int(rng.integers(20, 120)), n_vertices=int(rng.integers(3, 12)),
                       t_range=int(rng.integers(3, 40)))
    delta, k = int(rng.integers(0, 30)), int(rng.integers(1, 4))
    o = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.FAN_OUT | oracle.FAN_IN | oracle.SG | oracle.DEG_OUT |
                    oracle.DEG_IN, delta, 2, k)
    ou = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.SG | oracle.SG_UNORDERED, delta, 2, k)
    for prog, ref in ((P.FAN_OUT, o[0]), (P.FAN_IN, o[1]), (P.SG, o[2]), (P.DEG_OUT, o[3]), (P.DEG_IN, o[4]),
                      (P.SG_UNORDERED, ou[0])):
        np.testing.assert_array_equal(brute_program(g.src, g.dst, g.ts, prog, delta, k), ref.astype(np.uint64))


@pytest.mark.parametrize("seed", range(6))
def test_anchored_cycle_programs_count_each_cycle_once(seed):
    rng = np.random.default_rng(9200 + seed)
    g = W.random_small(seed + 920, n_edges=int(rng.integers(20, 100)), n_vertices=int(rng.integers(3, 9)),
                       t_range=int(rng.integers(5, 40)))
    delta = int(rng.integers(1, 40))
    first = oracle.count_cycles_first(g.src, g.dst, g.ts, g.n_vertices, delta, 5)
    for l in (2, 3, 4, 5):
        a = brute_program(g.src, g.dst, g.ts, P.cycle_anchored(l), delta, 1)
        assert int(a.sum()) == int(first[l])
        # and per edge: the oracle's credits of cycles found from that edge alone
        for e in np.flatnonzero(a)[:5]:
            c, _ = oracle.mine_range(g.src, g.dst, g.ts, g.n_vertices, int(e), int(e) + 1, oracle.CYC, delta, 5, 1)
            assert int(c[l - 2, e]) == int(a[e])
