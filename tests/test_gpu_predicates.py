"""GPU parity of the predicate chain (FP32 filter -> FP64 filter -> exact)
against the oracle's exact predicates, tuple by tuple, on the queries where
a wrong filter bound would show: near-ties with relative offsets 2^-20 ..
2^-60, the same scaled by 2^-80 .. 2^80, query points next to a vertex
(FP32 intermediates underflow) and plain random tuples.  The oracle's
predicates are pinned against exact rational determinants in
test_oracle.py on the same generators."""
import numpy as np
import pytest

import oracle
from tests import near_ties

pytestmark = pytest.mark.gpu


def _keys(q, npts, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(npts) * 5 + 2 for _ in range(q)]).astype(np.int64)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_insphere_signs_match_oracle(dtlib, dim, precision):
    q = near_ties.insphere_queries(dim, 6000, seed=100 + dim)
    keys = _keys(len(q), dim + 2, seed=7)
    print(f"[predicates] insphere {dim}d {precision}: {len(q)} tuples", flush=True)
    sign, stage = dtlib.predicates("insphere", q, keys, precision=precision)
    want = np.array([oracle.insphere(q[i], keys[i]) for i in range(len(q))], dtype=np.int8)
    bad = np.nonzero(sign != want)[0]
    assert len(bad) == 0, (bad[:5], q[bad[:1]], stage[bad[:5]])
    # the ties reach the exact stage; random tuples are decided by a filter
    assert (stage == 2).any()
    first = 0 if precision == "fp32" else 1
    assert (stage[3::4] == first).mean() > 0.9


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_orient_signs_match_oracle(dtlib, dim, precision):
    q = near_ties.orient_queries(dim, 6000, seed=200 + dim)
    print(f"[predicates] orient {dim}d {precision}: {len(q)} tuples", flush=True)
    sign, stage = dtlib.predicates("orient", q, precision=precision)
    want = np.array([oracle.orient(q[i]) for i in range(len(q))], dtype=np.int8)
    bad = np.nonzero(sign != want)[0]
    assert len(bad) == 0, (bad[:5], q[bad[:1]], stage[bad[:5]])
    assert (want == 0).any() and (stage == 2).any()


@pytest.mark.parametrize("dim", [2, 3])
def test_random_tuples_fp32_match_oracle(dtlib, dim):
    """Bulk random tuples: every FP32-certified sign is the exact sign."""
    rng = np.random.default_rng(5 + dim)
    q = rng.random((200_000, dim + 2, dim))
    keys = _keys(len(q), dim + 2, seed=3)
    print(f"[predicates] random insphere {dim}d", flush=True)
    sign, stage = dtlib.predicates("insphere", q, keys, precision="fp32")
    want = np.array([oracle.insphere(q[i], keys[i]) for i in range(len(q))], dtype=np.int8)
    assert np.array_equal(sign, want)
    assert (stage == 0).mean() > 0.99


def test_predicate_argument_errors(dtlib):
    with pytest.raises(ValueError):
        dtlib.predicates("insphere", np.zeros((4, 5, 3)), np.zeros((4, 4), np.int64))
    lib = dtlib.load()
    assert lib.dt_predicates(5, 3, 0, None, None, 1, None, None, None) == dtlib.DT_E_INVALID_ARG
    assert lib.dt_predicates(0, 4, 0, None, None, 1, None, None, None) == dtlib.DT_E_INVALID_ARG
    assert lib.dt_predicates(0, 3, 7, None, None, 1, None, None, None) == dtlib.DT_E_INVALID_ARG
    assert lib.dt_predicates(0, 3, 0, None, None, 1, None, None, None) == dtlib.DT_E_INVALID_ARG
    assert lib.dt_predicates(0, 3, 0, None, None, 0, None, None, None) == dtlib.DT_OK
