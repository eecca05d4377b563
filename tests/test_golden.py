"""Algorithm 3 on hand-derived cases (tests/golden/alg3_hand_derived.txt,
derivations and citations in the fixture): the oracle's blocking, and the
library's host analysis on the matrices whose Algorithm 2 pointer has those
closed forms."""
import os

import numpy as np
import pytest

from oracle import blocking

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    cases = []
    with open(os.path.join(HERE, "golden", "alg3_hand_derived.txt")) as fh:
        cur = None
        for line in fh:
            line = line.strip()
            if line.startswith("case "):
                f = line.split()
                kv = dict(x.split("=") for x in f[3:])
                cur = dict(name=f[1], kind=f[2], N=int(kv["N"]), step=int(kv["step"]),
                           max_num=int(kv["max_num"]), advance=int(kv["advance"]))
            elif line.startswith("ptr ") and cur is not None:
                cur["ptr"] = [int(x) for x in line.split()[1:]]
                cases.append(cur)
                cur = None
    return cases


CASES = _cases()


def _bp(kind, N):
    if kind == "tridiagonal":
        bp = np.zeros(N + 1, dtype=np.int64)
        bp[1:] = 3 * np.arange(1, N + 1) - 2
        return bp
    return np.arange(N + 1, dtype=np.int64) ** 2


def test_fixture_has_all_cases():
    assert sorted(c["name"] for c in CASES) == ["dense1000", "dense16", "tri1000", "tri1000_adv2"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_oracle_blocking_matches_hand_derivation(case):
    ptr = blocking.irregular_blocking(_bp(case["kind"], case["N"]), step=case["step"],
                                      max_num=case["max_num"], advance=case["advance"])
    assert ptr.tolist() == case["ptr"]


def _matrix(kind, N):
    if kind == "tridiagonal":
        r = np.concatenate([np.arange(N), np.arange(1, N), np.arange(N - 1)])
        c = np.concatenate([np.arange(N), np.arange(N - 1), np.arange(1, N)])
    else:
        r = np.repeat(np.arange(N), N)
        c = np.tile(np.arange(N), N)
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    rp = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp), c.astype(np.int32)


@pytest.mark.parametrize("case", [c for c in CASES if c["N"] * (c["N"] if c["kind"] == "dense" else 3) <= 10000],
                         ids=lambda c: c["name"])
def test_library_blocking_matches_hand_derivation(case):
    import paper_2512_04389_amd as slu
    rp, ci = _matrix(case["kind"], case["N"])
    h = slu.SparseLU(case["N"], rp, ci, step=case["step"], max_num=case["max_num"], advance=case["advance"])
    assert h.blocking().tolist() == case["ptr"]
    bp = h.blockptr()
    assert np.array_equal(bp, _bp(case["kind"], case["N"]))
    h.close()
