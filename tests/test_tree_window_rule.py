"""The rule the GPU's all-levels tree build rests on, checked on the CPU
against the oracle's recursive split (Sec. 2.3: cells split while they hold
more than leaf_size particles).

With the particles sorted by Morton key, the cell of level l holding
particle i has more than L particles exactly when some k in [i - L, i] has
keys k and k + L sharing their first l octal digits; so i's leaf is at level
d(i) = 1 + max c(k) over that window (c(k): common leading levels of keys k
and k + L), the cells that start at i are those of levels cp(i) + 1 .. d(i)
(cp(i): common levels of keys i - 1 and i) and the runs that end at i those
of levels cp(i + 1) + 1 .. d(i).  Building every level from these per-particle
ranges must give the oracle's tree: same cells, bounds, levels, prefixes and
leaf flags.
"""
import numpy as np
import pytest
from scipy.ndimage import maximum_filter1d

from oracle import oracle as O
from paper_1712_10116_amd import workloads as W

MAXL = 21


def _keys(pos):
    lo, hi = pos.min(axis=1), pos.max(axis=1)
    c = 0.5 * (lo + hi)
    side = float((hi - lo).max()) or 1.0
    q = np.floor((pos - (c - 0.5 * side)[:, None]) * (2097152.0 / side))
    q = np.minimum(np.where(q >= 0, q, 0.0), float((1 << MAXL) - 1)).astype(np.uint64)
    key = np.zeros(pos.shape[1], dtype=np.uint64)
    for b in range(MAXL):
        for ax, sh in ((0, 2), (1, 1), (2, 0)):
            key |= ((q[ax] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + sh)
    return key


def _common(a, b):
    x = a ^ b
    bl = np.array([int(v).bit_length() for v in x], dtype=np.int64)
    return np.where(x == 0, MAXL, (64 - bl - 1) // 3)


def _rule_tree(key, L):
    n = key.size
    c = np.full(n, -1, dtype=np.int64)
    if n > L:
        c[: n - L] = _common(key[: n - L], key[L:])
    # window max over [i - L, i]
    m = maximum_filter1d(c, size=L + 1, origin=L // 2 if (L + 1) % 2 else (L + 1) // 2 - 1,
                         mode="constant", cval=-1)
    d = np.where(m < 0, 0, np.minimum(MAXL, m + 1))
    cp = np.zeros(n, dtype=np.int64)
    cp[1:] = _common(key[:-1], key[1:])
    lo = cp + 1
    lo[0] = 1
    lo2 = np.zeros(n, dtype=np.int64)
    lo2[:-1] = cp[1:] + 1
    lev, beg, end, leaf = [0], [0], [n], [int(d[0] == 0)]
    for l in range(1, MAXL + 1):
        s = np.nonzero((lo <= l) & (l <= d))[0]
        e = np.nonzero((lo2 <= l) & (l <= d))[0] + 1
        assert s.size == e.size
        lev += [l] * s.size
        beg += s.tolist()
        end += e.tolist()
        leaf += (d[s] <= l).astype(int).tolist()
    return np.array(lev), np.array(beg), np.array(end), np.array(leaf), d


def _window_max_direct(c, L):
    return np.array([c[max(0, i - L): i + 1].max() for i in range(c.size)])


@pytest.mark.parametrize("case", ["uniform3000_16", "uniform20000_96", "uniform20000_8",
                                  "plummer4096_16", "clustered4000_16", "tiny_700_64"])
def test_window_rule_builds_the_oracle_tree(case):
    rng = np.random.default_rng(11)
    if case.startswith("uniform"):
        n, L = (int(x) for x in case[7:].split("_"))
        pos = W.uniform_sphere(n, seed=int(rng.integers(1 << 30)))[0]
    elif case.startswith("plummer"):
        pos, L = W.config(0, n=4096)[0], 16
    elif case.startswith("clustered"):
        # a tight clump (deep levels) and exact duplicates (keys equal to the last digit)
        pos = rng.normal(size=(3, 4000))
        pos[:, :1500] = 1e-7 * rng.normal(size=(3, 1500))
        pos[:, 1500:1600] = pos[:, 1600:1700]
        L = 16
    else:
        pos, L = W.uniform_sphere(700, seed=3)[0], 64
    pos = np.ascontiguousarray(pos)
    key = _keys(pos)
    perm = np.argsort(key, kind="stable")
    skey = key[perm]
    lev, beg, end, leaf, d = _rule_tree(skey, L)
    t = O.Tree(pos, p=2, theta=0.5, eps=0.01, leaf_size=L, kernel=O.PLUMMER)
    ex = t.export()
    np.testing.assert_array_equal(ex["perm"], perm)
    o1, o2 = np.lexsort((lev, beg)), np.lexsort((ex["level"], ex["begin"]))
    np.testing.assert_array_equal(lev[o1], ex["level"][o2])
    np.testing.assert_array_equal(beg[o1], ex["begin"][o2])
    np.testing.assert_array_equal(end[o1], ex["end"][o2])
    np.testing.assert_array_equal(leaf[o1], ex["is_leaf"][o2])
    pre = np.array([int(skey[b]) >> (3 * (MAXL - l)) if l else 0 for l, b in zip(lev, beg)],
                   dtype=np.uint64)
    np.testing.assert_array_equal(pre[o1], ex["prefix"][o2])


def test_window_max_filter_alignment():
    """The filter above takes the maximum over [i - L, i] exactly."""
    rng = np.random.default_rng(3)
    c = rng.integers(-1, 21, size=500)
    for L in (1, 2, 7, 16, 63, 96):
        m = maximum_filter1d(c, size=L + 1, origin=L // 2 if (L + 1) % 2 else (L + 1) // 2 - 1,
                             mode="constant", cval=-1)
        np.testing.assert_array_equal(m, _window_max_direct(c, L))
