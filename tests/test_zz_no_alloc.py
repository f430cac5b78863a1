"""pthr_autotune_noalloc (the allocation-free variant of pthr_autotune)
against pthr_autotune on the same inputs, two calls in a row (the second on a
smaller input), and its size limit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2605_25872_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(L, S, NR, NT, NER, precision, seed):
    from paper_2605_25872_amd import pthr
    J = inputs.couplings(L, S, seed=seed)
    T = inputs.temperatures(0.3, 1.6, NT)
    ctxs = []
    for _ in range(2):
        g = pthr.Pthr(L, S, NR, NT, NER, 10, 24, precision, "acu", 1.0, seed)
        g.init_samples(J, T)
        ctxs.append(g)
    o = oracle.Oracle(L, S, NR, NT, NER, 10, 24, oracle.FP64 if precision == "fp64" else oracle.FP32,
                      oracle.ACU, 1.0, seed)
    o.init(J, T)
    return o, ctxs[0], ctxs[1]


def _same(a, b):
    assert np.array_equal(a.read_spins(), b.read_spins())
    pa, pb = a.read_pt(), b.read_pt()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    assert a.counters() == b.counters()


@pytest.mark.parametrize("case", [(8, 6, 4, 10, 4, "fp32", 3), (6, 3, 2, 7, 3, "fp64", 4)])
def test_noalloc_autotune_matches_workspace_autotune(case):
    """The two calls in a row run on the library's one static workspace: a
    larger state first, then a smaller one.  Each variant leaves the state
    untouched and picks a valid schedule; since every schedule gives the same
    bits, the runs that follow are identical to each other and to the
    oracle."""
    L, S, NR, NT, NER, prec, seed = case
    print(f"[no-alloc] L={L} S={S} {prec}", file=sys.stderr, flush=True)
    o, a, b = _pair(L, S, NR, NT, NER, prec, seed)
    o.run(1)
    a.run(1)
    b.run(1)
    ms_a = a.autotune(1)
    ms_b = b.autotune_noalloc(1)
    assert ms_a > 0 and ms_b > 0
    _same(a, b)
    sa, sb = a.schedule(), b.schedule()
    assert sb.graph_window == sa.graph_window
    assert sb.clone_split in (1, 2, 4) and sb.threads_per_sample * sb.clone_split <= 1024
    o.run(2)
    a.run(2)
    b.run(2)
    _same(a, b)
    assert np.array_equal(b.read_spins(), o.spins)
    assert np.array_equal(b.read_pt()["clone_at"], o.clone_at)


def test_noalloc_autotune_rejects_a_state_beyond_its_workspace():
    from paper_2605_25872_amd import pthr
    w = inputs.WORKLOADS["l16_fp32"]
    g = pthr.Pthr(16, 512, 4, 36, 4, 10, 240, "fp32", "acu", 1.0, 1)
    assert g.state_bytes > 64 << 20
    g.init_samples(w.couplings(512), w.temperatures())
    with pytest.raises(pthr.PthrError, match="static workspace"):
        g.autotune_noalloc(1)
