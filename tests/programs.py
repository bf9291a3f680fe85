"""Stage-cell programs of the paper's patterns (amlm_cell field dicts),
shared by the CPU and GPU tests of the interpreter."""
U, V = 0, 1
FOR_OUT, FOR_IN, PROBE = 0, 1, 2
WINDOW, AFTER = 0, 1
THROUGH, BEFORE = 0, 1
SUM, AT_LEAST, AT_LEAST_K = 0, 1, 2


def C(op, node, peer=0, tlo=WINDOW, tref=0, thi=THROUGH, skip=(), distinct=False, agg=SUM, threshold=0):
    return dict(op=op, node=node, peer=peer, tlo=tlo, tref=tref, thi=thi, skip=tuple(skip),
                distinct=int(distinct), agg=agg, threshold=threshold)


# the fixed kernels' columns, re-expressed as stage cells
FAN_OUT = [C(FOR_OUT, U)]
FAN_IN = [C(FOR_IN, V)]
DEG_OUT = [C(FOR_OUT, U, distinct=True)]
DEG_IN = [C(FOR_IN, V, distinct=True)]
# SG_k: senders s into u before t (skip v, each once) with at least k
# intermediates m: s's first edge to m in the window, then an m -> v edge
# after it, up to t (u itself qualifies through the anchor)
SG = [C(FOR_IN, U, thi=BEFORE, skip=(V,), distinct=True, agg=AT_LEAST_K),
      C(FOR_OUT, 2, thi=BEFORE, distinct=True, agg=AT_LEAST, threshold=1),
      C(PROBE, 3, peer=V, tlo=AFTER, tref=1)]
SG_UNORDERED = [SG[0], SG[1], C(PROBE, 3, peer=V)]


def cycle_anchored(l):
    """l-cycles whose last edge is the anchor: a path v -> ... -> u of l - 1
    edges with rising times inside [t - delta, t), on fresh vertices."""
    if l == 2:
        return [C(PROBE, V, peer=U, thi=BEFORE)]
    cells = [C(FOR_OUT, V, thi=BEFORE, skip=(U, V))]
    for i in range(1, l - 2):
        cells.append(C(FOR_OUT, 1 + i, tlo=AFTER, tref=i - 1, thi=BEFORE, skip=(U, V) + tuple(range(2, 2 + i))))
    cells.append(C(PROBE, l - 1, peer=U, tlo=AFTER, tref=l - 3, thi=BEFORE))
    return cells


def random_program(rng):
    """A random valid program of 1..4 cells."""
    n = int(rng.integers(1, 5))
    cells = []
    for i in range(n):
        bound = 2 + i
        last = i + 1 == n
        op = int(rng.integers(0, 3)) if last else int(rng.integers(0, 2))
        tlo = AFTER if i > 0 and cells[-1]["op"] != PROBE and rng.random() < 0.5 else WINDOW
        skip = tuple(b for b in range(bound) if rng.random() < 0.3)
        cells.append(C(op, int(rng.integers(0, bound)), peer=int(rng.integers(0, bound)), tlo=tlo,
                       tref=int(rng.integers(0, i)) if tlo == AFTER else 0, thi=int(rng.integers(0, 2)),
                       skip=skip, distinct=bool(rng.random() < 0.5), agg=int(rng.integers(0, 3)),
                       threshold=int(rng.integers(1, 4))))
    return cells
