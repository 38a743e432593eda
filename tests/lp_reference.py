"""Plain numpy statement of the label-propagation rule that bc_partition_lp documents
(test infrastructure; shares no code with the library): used to check the device
partitioner label for label."""
import numpy as np


def splitmix64(x):
    """SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) of counter x."""
    x = np.asarray(x, np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return x ^ (x >> np.uint64(31))


def label_propagation(g, cap, rounds, seed):
    """(part [n] int32, k): every node starts alone; per round the nodes whose hash of
    (seed, round, node) is odd move to the label most common among their neighbours
    among labels held by fewer than cap nodes (cap 0: any), when strictly more common
    than their own, ties to the smallest label; sizes recounted per round; labels
    renumbered in increasing order."""
    n = g.n
    lab = np.arange(n, dtype=np.int64)
    size = np.ones(n, np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    dst = np.asarray(g.col, np.int64)
    vid = np.arange(n, dtype=np.uint64)
    for r in range(rounds):
        h = splitmix64(np.uint64(seed) ^ (np.uint64(r) << np.uint64(32)) ^ vid)
        active = (h & np.uint64(1)) == np.uint64(1)
        uk, cnt = np.unique(src * n + lab[dst], return_counts=True)
        kv, kl = uk // n, uk % n
        is_cur = kl == lab[kv]
        c0 = np.zeros(n, np.int64)
        c0[kv[is_cur]] = cnt[is_cur]
        ok = ~is_cur
        if cap > 0:
            ok &= size[kl] < cap
        kv, kl, cnt = kv[ok], kl[ok], cnt[ok]
        order = np.lexsort((kl, -cnt, kv))
        kv, kl, cnt = kv[order], kl[order], cnt[order]
        first = np.ones(kv.size, bool)
        first[1:] = kv[1:] != kv[:-1]
        bv, bl, bc = kv[first], kl[first], cnt[first]
        move = active[bv] & (bc > c0[bv])
        new = lab.copy()
        new[bv[move]] = bl[move]
        lab = new
        size = np.bincount(lab, minlength=n)
    used = np.nonzero(size)[0]
    ids = np.full(n, -1, np.int64)
    ids[used] = np.arange(used.size)
    return ids[lab].astype(np.int32), int(used.size)
