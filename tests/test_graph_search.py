"""The two searches over the sample's Delaunay graph, checked on the CPU
against the oracle (they are what the assignment and the Voronoi border
test of the sample divide run on the GPU; the GPU kernels themselves are
compared with the oracle in the gpu tests).

1. Nearest sample by descent: the squared distance to a point x, taken
   over the samples, is the lifted height |s|^2 less an affine function of
   s, and the DT is the lower hull of the lifted samples, so every set
   {s : |x - s|^2 <= L} is connected through Delaunay edges.  A greedy
   descent under the key (fl(d^2), id), followed by a search of the samples
   whose key is within 1e-9 of the final one, must give the oracle's key
   minimum over all samples, ties included.
2. The Voronoi walk of the border test: a simplex of T_i whose circumball
   the walk does not flag holds no point of another partition, so every
   simplex of T_i that is not in DT(P) is flagged.  The same holds for the
   clearance prefilter in front of it: a simplex is settled without the walk
   when a vertex's least distance to a bisector of its own sample and a
   foreign sample exceeds 2r (the GPU uses a lower bound of that distance,
   which settles fewer)."""
import numpy as np

import oracle
from paper_1902_07554_amd import inputs


def _key(x, q, qid):
    d = 0.0
    for a in range(len(x)):
        t = x[a] - q[a]
        d = t * t if a == 0 else d + t * t
    return d, int(qid)


def _sample_graph(p, n, eta, seed):
    sid = oracle.sample_ids(n, eta, seed)
    S = p[sid]
    rows = oracle.delaunay(S, sid)                 # rows of sample ids
    loc = np.searchsorted(sid, rows)               # sid is ascending
    adj = [[] for _ in range(eta)]
    for a, b in oracle.graph_edges(loc):
        adj[a].append(int(b))
        adj[b].append(int(a))
    return sid, S, [sorted(x) for x in adj]


def _descend(x, S, sid, adj, t):
    kt = _key(x, S[t], sid[t])
    while True:
        best, kb = t, kt
        for w in adj[t]:
            kw = _key(x, S[w], sid[w])
            if kw < kb:
                best, kb = w, kw
        if best == t:
            return t, kt
        t, kt = best, kb


def _nearest_by_descent(x, S, sid, adj, start):
    t, kt = _descend(x, S, sid, adj, start)
    lim = kt[0] * (1.0 + 1e-9)
    seen, todo, best, kb = {t}, [t], t, kt
    while todo:
        u = todo.pop()
        for w in adj[u]:
            if w in seen:
                continue
            kw = _key(x, S[w], sid[w])
            if kw[0] <= lim:
                seen.add(w)
                todo.append(w)
                if kw < kb:
                    best, kb = w, kw
    return best


def test_descent_gives_the_key_minimum():
    rng = np.random.default_rng(4)
    # lattices give exact ties; scaled by 0.1 and shifted, ties within rounding
    cases = [inputs.make("uniform", 3000, 3, seed=2), inputs.make("normal", 3000, 2, seed=3),
             inputs.lattice(9, 3, seed=4), inputs.lattice(30, 2, seed=5),
             inputs.lattice(9, 3, seed=4) * 0.1 + 0.37, inputs.lattice(40, 2, seed=6) * 0.1 + 0.37]
    for p in cases:
        n = len(p)
        eta = max(p.shape[1] + 2, n // 30)
        sid, S, adj = _sample_graph(p, n, eta, seed=7)
        want = oracle.nearest_sample(p, S, sid)
        got = np.array([_nearest_by_descent(p[i], S, sid, adj, int(rng.integers(eta)))
                        for i in range(n)])
        assert np.array_equal(got, want)


def _circumball(v):
    a = v[1:] - v[0]
    rhs = 0.5 * np.einsum("ij,ij->i", a, a)
    c = np.linalg.solve(a, rhs)
    return v[0] + c, float(np.sqrt(c @ c))


def _walk_flags(x_c, r, S, sid, part, adj, me, t, cap=16):
    """True when the walk flags the ball (centre x_c, radius r) of a simplex
    of partition `me`, starting from the own sample t."""
    def d2(s):
        q = x_c - S[s]
        return float(q @ q)

    t, _ = _descend(x_c, S, sid, adj, t)
    if part[t] != me:
        return True

    def reach(u, du, w, dw):
        gap = float(np.linalg.norm(S[w] - S[u]))
        return dw - du <= 2.0 * gap * r + 2e-12 * (du + dw + 2.0 * r * r)

    dt = d2(t)
    vis, head = [t], 0
    while head < len(vis):
        u = vis[head]
        head += 1
        du = d2(u)
        for w in adj[u]:
            if w in vis:
                continue
            dw = d2(w)
            if reach(u, du, w, dw) and (u == t or reach(t, dt, w, dw)):
                if part[w] != me or len(vis) == cap:
                    return True
                vis.append(w)
    return False


def test_voronoi_walk_flags_every_non_delaunay_simplex():
    p = inputs.make("bubbles", 2500, 3, seed=6)
    n, k = len(p), 6
    eta = 80
    sid, S, adj = _sample_graph(p, n, eta, seed=9)
    part = np.arange(eta) * k // eta               # contiguous in id order
    near = oracle.nearest_sample(p, S, sid)
    pid = part[near]
    full = {tuple(r) for r in oracle.delaunay(p)}
    # clearance of every point from the foreign cells, over all samples
    clear = np.empty(n)
    for j in range(n):
        t = near[j]
        fs = np.nonzero(part != part[t])[0]
        ds = np.einsum("ij,ij->i", p[j] - S[fs], p[j] - S[fs])
        dt = float((p[j] - S[t]) @ (p[j] - S[t]))
        clear[j] = np.min((ds - dt) / (2.0 * np.linalg.norm(S[fs] - S[t], axis=1)))
    settled = 0
    flagged = missed = total = outside = 0
    for i in range(k):
        mine = np.nonzero(pid == i)[0]
        if len(mine) < 4:
            continue
        for row in oracle.delaunay(p[mine], mine):
            v = p[row]
            c, r = _circumball(v)
            r *= 1.0 + 1e-9
            # start from the vertex sample nearest to the centre
            t = min((int(near[j]) for j in row), key=lambda s: float((c - S[s]) @ (c - S[s])))
            f = _walk_flags(c, r, S, sid, part, adj, i, t)
            flagged += f
            total += 1
            pre = max(clear[j] for j in row) > 2.0 * r
            settled += pre
            if tuple(row) not in full:
                outside += 1
                missed += (not f) + pre
    # the case has simplices to catch, and the walk does not flag everything
    assert outside > 0 and flagged < total and settled > 0
    assert missed == 0


def _list_clearance(p, S, part, near, ml):
    """The clearance from a short list per sample: the ml foreign samples
    of smallest squared distance to t rounded to FP32 (keys below the
    (ml+1)-th smallest key), and rho_t, half the least distance of the
    foreign samples not listed."""
    ns = len(S)
    lists, rho = [], np.full(ns, np.inf)
    for t in range(ns):
        fs = np.nonzero(part != part[t])[0]
        e = S[fs] - S[t]
        g2 = e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1] + e[:, 2] * e[:, 2]
        if len(fs) <= ml:
            lists.append(fs)
            continue
        keys = g2.astype(np.float32)
        thr = np.sort(keys)[ml]
        take = keys < thr
        assert take.sum() <= ml
        lists.append(fs[take])
        rho[t] = 0.5 * float(np.sqrt(g2[~take].min()))
    out = np.empty(len(p))
    from_rho = 0
    for j in range(len(p)):
        t = near[j]
        dt = float((p[j] - S[t]) @ (p[j] - S[t]))
        rt = np.sqrt(dt)
        f = rho[t] * (1.0 - 1e-9) - rt * (1.0 + 1e-9)
        f_rho = f
        for s in lists[t]:
            ds = float((p[j] - S[s]) @ (p[j] - S[s]))
            gap = float(np.linalg.norm(S[s] - S[t]))
            f = min(f, (ds - dt - 1e-12 * (ds + dt)) / (2.0 * gap))
        from_rho += f == f_rho
        out[j] = f
    return out, from_rho


def test_listed_clearance_is_a_lower_bound():
    """The border test's clearance of a point from the foreign Voronoi
    cells, taken from its sample's list of nearest foreign samples and the
    distance bound for the others, never exceeds the clearance over all
    foreign samples, and with a short list the bound for the others decides
    some points."""
    p = inputs.make("bubbles", 3000, 3, seed=8)
    eta, k = 96, 8
    sid, S, adj = _sample_graph(p, len(p), eta, seed=4)
    part = np.arange(eta) * k // eta
    near = oracle.nearest_sample(p, S, sid)
    exact = np.empty(len(p))
    for j in range(len(p)):
        t = near[j]
        fs = np.nonzero(part != part[t])[0]
        ds = np.einsum("ij,ij->i", p[j] - S[fs], p[j] - S[fs])
        dt = float((p[j] - S[t]) @ (p[j] - S[t]))
        exact[j] = np.min((ds - dt) / (2.0 * np.linalg.norm(S[fs] - S[t], axis=1)))
    for ml in (2, 6, 32):
        got, from_rho = _list_clearance(p, S, part, near, ml)
        assert np.all(got <= exact + 1e-12 * np.abs(exact))
        if ml <= 6:
            assert from_rho > 0
    # with the library's list length the bound is nearly the exact one
    got, _ = _list_clearance(p, S, part, near, 32)
    assert np.mean(got >= exact - 1e-6 * np.abs(exact)) > 0.9
