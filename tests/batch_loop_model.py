"""Lane-level CPU model of the fast batching path (the graph kernel and the register-resident
loop kernel), written after the HIP code: 64 lanes x S register slots, ballots as bit masks, the
leader cache in scalars.  Where the kernel does several lanes' work at once (the finished lanes'
group count-downs, the lane-parallel convoy stores) the model does it lane by lane, which gives
the same state.  Test infrastructure: it lets the CPU suite
check the fast path's logic (leader runs, holes, in-place successors, compaction, the
ready-set bound) against the oracle without a GPU; the GPU tests check the kernels themselves.
"""
import numpy as np

INV = 0xFFFFFFFF; MY = 0xC00001FF; MX = 0xC0000000 | (0x1FF << 15); M32 = 0xFFFFFFFF
W64 = 64
def delta_of(d): return [1 << 15, (-(1 << 15)) & M32, 1, 0xFFFFFFFF][d]
def entry_of(m):
    sx, sy, dx, dy = m & 0xFF, (m >> 8) & 0xFF, (m >> 16) & 0xFF, m >> 24
    if sx != dx:
        d = 0 if dx > sx else 1
        return (d << 30) | (sx << 15) | sy, (d << 30) | (dx << 15) | sy, ((((2 if dy > sy else 3) << 30) | (dx << 15) | dy) if dy != sy else INV)
    d = 2 if dy > sy else 3
    return (d << 30) | (sx << 15) | sy, (d << 30) | (dx << 15) | dy, INV
def ballot(v): return int(sum((1 << l) for l in range(64) if v[l]))
def ffs(m): return (m & -m).bit_length() - 1
def fls(m): return m.bit_length() - 1
def popc(m): return bin(m).count('1')
def range_mask(lo, hi):
    if hi < lo or hi < 0 or lo > 63: return 0
    lo = max(lo, 0); hi = min(hi, 63)
    return ((1 << (hi + 1)) - 1) & ~((1 << lo) - 1)

class R:
    def __init__(s, S):
        s.S = S
        s.c = [[INV] * 64 for _ in range(S)]; s.e = [[INV] * 64 for _ in range(S)]
        s.n = [[INV] * 64 for _ in range(S)]; s.k = [[INV] * 64 for _ in range(S)]; s.vm = [0] * S

def merge_insert(Rr, c0, e0, n0, k0, scr):
    S = Rr.S
    total = 1 + sum(popc(v) for v in Rr.vm)
    if total > 64 * S: return False
    base = 0; nlt = 0
    for s in range(S):
        v = Rr.vm[s]
        nlt += popc(ballot([Rr.k[s][l] < k0 for l in range(64)]) & v)
        for l in range(64):
            if (v >> l) & 1:
                r = base + popc(v & ((1 << l) - 1)) + (1 if Rr.k[s][l] > k0 else 0)
                scr[r] = (Rr.c[s][l], Rr.e[s][l], Rr.n[s][l], Rr.k[s][l])
        base += popc(v)
    scr[nlt] = (c0, e0, n0, k0)
    for s in range(S):
        for l in range(64):
            p = s * 64 + l
            q = scr[p] if p < total else (INV, INV, INV, INV)
            Rr.c[s][l], Rr.e[s][l], Rr.n[s][l], Rr.k[s][l] = q
        Rr.vm[s] = ballot([s * 64 + l < total for l in range(64)])
    return True

def insert_ready(Rr, Gd, b, g, ps, pl, st, scr):
    S = Rr.S
    c0, e0, n0 = entry_of(Gd['mv'][b]); k0 = (b << 10) | g
    lo, hi = -1, 64 * S
    for s in range(S):
        v = Rr.vm[s]
        if v:
            lt = ballot([Rr.k[s][l] < k0 for l in range(64)]) & v; gt = v & ~lt
            if lt: lo = s * 64 + fls(lt)
            if gt and hi == 64 * S: hi = s * 64 + ffs(gt)
    pos = -1
    if ps >= 0:
        pp = ps * 64 + pl
        if lo < pp < hi and not ((Rr.vm[ps] >> pl) & 1): pos = pp
    if pos < 0 and hi - lo > 1:
        for s in range(S):
            if pos >= 0: continue
            holes = ~Rr.vm[s] & range_mask(lo + 1 - s * 64, hi - 1 - s * 64) & ((1 << 64) - 1)
            if holes: pos = s * 64 + ffs(holes)
    if pos >= 0:
        s, l = divmod(pos, 64)
        Rr.c[s][l], Rr.e[s][l], Rr.n[s][l], Rr.k[s][l] = c0, e0, n0, k0; Rr.vm[s] |= 1 << l
        st['inplace' if pos == (ps * 64 + pl if ps >= 0 else -9) else 'hole'] += 1
        return True
    st['moved'] = True; st['merge'] += 1
    return merge_insert(Rr, c0, e0, n0, k0, scr)

def release_move(Rr, Gd, b, g, ps, pl, st, scr, grem, gpend, pend):
    ok = True
    code = Gd['nx'][b]; kind = code >> 14
    if kind == 1: ok &= insert_ready(Rr, Gd, b + (code & 16383), g, ps, pl, st, scr)
    elif kind == 2:
        for nxm in Gd['succ'][b]:
            old = pend[nxm]; pend[nxm] -= 1
            if old == 1: ok &= insert_ready(Rr, Gd, nxm, g, ps, pl, st, scr)
    left = grem[g]; grem[g] -= 1
    if left == 1:
        for h in sorted(Gd['gw'][g]):
            old = gpend[h]; gpend[h] -= 1
            if old == 1:
                for hb in Gd['heads'][h]: ok &= insert_ready(Rr, Gd, hb, h, -1, -1, st, scr)
    return ok

def find_leader(Rr):
    for s in range(Rr.S):
        if Rr.vm[s]:
            l = ffs(Rr.vm[s]); return s, l, Rr.c[s][l], Rr.e[s][l], Rr.n[s][l], Rr.k[s][l]
    return -1, 0, INV, INV, INV, INV

def axis_pos(c, horiz):
    return (c >> 15) & 0x1FF if horiz else c & 0x1FF


def loop(Gd, S, flags):
    """Alg. 3 over the graph Gd with 64*S register positions, as the loop kernel runs it: one batch
    per trip (the leader alone, or the leader and the moves on its row or column that step its
    way), then the same batch repeated -- the convoy -- until a member ends its leg or a waiting
    move reaches the line that sweeps with the leader."""
    K, G = Gd['K'], Gd['G']
    T = sum(abs(((m >> 16) & 0xFF) - (m & 0xFF)) + abs((m >> 24) - ((m >> 8) & 0xFF)) for m in Gd['mv'])
    grem = [Gd['goff'][g + 1] - Gd['goff'][g] for g in range(G)]
    gpend = list(Gd['gpend']); pend = list(Gd['pend'])
    scr = [None] * (64 * S)
    Rr = R(S)
    ents = []
    for g in range(G):
        if gpend[g] == 0:
            for b in Gd['heads'][g]:
                c, e, n = entry_of(Gd['mv'][b]); ents.append((c, e, n, (b << 10) | g))
    assert len(ents) <= 64 * S
    for p, q in enumerate(ents):
        s, l = divmod(p, 64); Rr.c[s][l], Rr.e[s][l], Rr.n[s][l], Rr.k[s][l] = q; Rr.vm[s] |= 1 << l
    st = dict(inplace=0, hole=0, merge=0, moved=False, trips=0, repeats=0, bulk=0)
    alive = K; out = 0; nb = 0; steps = []; boff = [0]
    ls, ll, lc, le, ln, lk = find_leader(Rr)
    while alive > 0:
        if nb >= T or ls < 0: raise RuntimeError('err')
        st['trips'] += 1
        d1 = lc >> 30; delta = delta_of(d1); lbit = 1 << ll
        horiz = d1 < 2
        acc = [0] * S; found = False; along = False
        if flags == 2:
            acc = list(Rr.vm); found = True
        else:
            ky, kx = lc & MY, lc & MX
            use_row = flags != 1 or d1 < 2; use_col = flags != 1 or d1 >= 2
            row = False
            for s in range(S):
                if Rr.vm[s] and not found:
                    mr = ballot([(Rr.c[s][l] & MY) == ky for l in range(64)]) if use_row else 0
                    mc = ballot([(Rr.c[s][l] & MX) == kx for l in range(64)]) if use_col else 0
                    if s == ls: mr &= ~lbit; mc &= ~lbit
                    if mr | mc:
                        found = True; row = bool((mr >> ffs(mr | mc)) & 1)
            if found:
                along = row == horiz
                for s in range(S):
                    if Rr.vm[s]:
                        acc[s] = ballot([((Rr.c[s][l] & (MY if row else MX)) == (ky if row else kx)) for l in range(64)])
            acc[ls] |= lbit
        # first member after the leader (along batches): its key bounds the sweeping-line blockers
        amin = None
        if found and along:
            for s in range(S):
                m = acc[s] & ~(lbit if s == ls else 0)
                if m and amin is None: amin = Rr.k[s][ffs(m)]
        # ---- the batch: members step in index order
        base = 0; arr = [0] * S
        for s in range(S):
            a = acc[s]
            if a:
                for l in range(64):
                    if (a >> l) & 1:
                        assert out + base + popc(a & ((1 << l) - 1)) == len(steps)
                        steps.append(Rr.c[s][l])
                        Rr.c[s][l] = (Rr.c[s][l] + (delta_of(Rr.c[s][l] >> 30) if flags == 2 else delta)) & M32
                arr[s] = ballot([((a >> l) & 1) and Rr.c[s][l] == Rr.e[s][l] for l in range(64)])
                base += popc(a)
        out += base; nb += 1; boff.append(out); lc = (lc + delta) & M32
        # ---- the convoy: repeats of the same batch
        if not any(arr):
            tv = [1 << 20] * 64
            for s in range(S):
                a = acc[s]
                if a:
                    for l in range(64):
                        if (a >> l) & 1:
                            c, e = Rr.c[s][l], Rr.e[s][l]
                            h = (c >> 30) < 2
                            rem = abs(axis_pos(e, h) - axis_pos(c, h))
                            tv[l] = min(tv[l], rem)
            if flags == 0:
                p1 = axis_pos(lc, horiz)                      # the leader's new position
                for s in range(S):
                    if Rr.vm[s]:
                        for l in range(64):
                            if (Rr.vm[s] >> l) & 1 and not (acc[s] >> l) & 1:
                                c = Rr.c[s][l]
                                if (c >> 30) != d1: continue
                                if along and Rr.k[s][l] > amin: continue
                                # on the sweeping line: column for a horizontal leg, row for a vertical one
                                p = axis_pos(c, horiz)
                                t = ((p1 - p) if (d1 & 1) else (p - p1)) & M32
                                if t < tv[l]: tv[l] = t
            ts = min(tv)
            if ts > 0:
                st['repeats'] += ts; st['bulk'] += 1
                for j in range(ts):
                    for s in range(S):
                        a = acc[s]
                        for l in range(64):
                            if (a >> l) & 1:
                                dl = delta_of(Rr.c[s][l] >> 30) if flags == 2 else delta
                                steps.append((Rr.c[s][l] + j * dl) & M32)
                    boff.append(out + (j + 1) * base)
                out += ts * base; nb += ts; lc = (lc + ts * delta) & M32
                for s in range(S):
                    a = acc[s]
                    if a:
                        for l in range(64):
                            if (a >> l) & 1:
                                dl = delta_of(Rr.c[s][l] >> 30) if flags == 2 else delta
                                Rr.c[s][l] = (Rr.c[s][l] + ts * dl) & M32
                        arr[s] = ballot([((a >> l) & 1) and Rr.c[s][l] == Rr.e[s][l] for l in range(64)])
        # ---- legs ended: turn or finish
        done = [0] * S; ndone = 0; ldone = False
        for s in range(S):
            if arr[s]:
                me = [(arr[s] >> l) & 1 for l in range(64)]
                turn = [me[l] and Rr.n[s][l] != INV for l in range(64)]
                done[s] = ballot([me[l] and not turn[l] for l in range(64)])
                for l in range(64):
                    if turn[l]:
                        Rr.c[s][l] = (Rr.c[s][l] & 0x3FFFFFFF) | (Rr.n[s][l] & 0xC0000000); Rr.e[s][l] = Rr.n[s][l]; Rr.n[s][l] = INV
                if s == ls and (arr[s] >> ll) & 1:
                    if (done[s] >> ll) & 1: ldone = True
                    else: lc = (lc & 0x3FFFFFFF) | (ln & 0xC0000000); le = ln; ln = INV
                ndone += popc(done[s])
        if ndone == 0:
            assert Rr.c[ls][ll] == lc and Rr.e[ls][ll] == le, 'leader cache'
            continue
        dk = [list(Rr.k[s]) for s in range(S)]
        for s in range(S):
            if done[s]:
                for l in range(64):
                    if (done[s] >> l) & 1: Rr.c[s][l] = INV; Rr.k[s][l] = INV
                Rr.vm[s] &= ~done[s]
        alive -= ndone
        st['moved'] = False; ok = True
        for s in range(S):
            m = done[s]
            while m:
                l = ffs(m); m &= m - 1
                kk = dk[s][l]
                ok &= release_move(Rr, Gd, kk >> 10, kk & 0x3FF, s, l, st, scr, grem, gpend, pend)
        if not ok: raise RuntimeError('overflow')
        if ldone or st['moved']: ls, ll, lc, le, ln, lk = find_leader(Rr)
        else:
            assert Rr.c[ls][ll] == lc and Rr.e[ls][ll] == le and Rr.n[ls][ll] == ln, 'leader cache'
    return np.array(boff, np.uint32), np.array(steps, np.uint32), st


def paths_meet(p, q):
    """Do the H-then-V paths of moves p, q = (sx, sy, dx, dy) share a trap (paths_meet)?"""
    def spans(v, a, b): return min(a, b) <= v <= max(a, b)
    def overlap(a1, b1, a2, b2): return max(min(a1, b1), min(a2, b2)) <= min(max(a1, b1), max(a2, b2))
    psx, psy, pdx, pdy = p; qsx, qsy, qdx, qdy = q
    return ((psy == qsy and overlap(psx, pdx, qsx, qdx)) or (spans(qdx, psx, pdx) and spans(psy, qsy, qdy))
            or (spans(pdx, qsx, qdx) and spans(qsy, psy, pdy)) or (pdx == qdx and overlap(psy, pdy, qsy, qdy)))


def pred_add(ps, a, mvs, reduce=True):
    """Add in-group predecessor a to the list ps as pred_add does: members whose paths meet a's
    and that come before a are dropped, a is not added when a later member's path meets it.
    Returns True when a needed member did not fit (8 at most).  reduce=False keeps every
    distinct member, without that limit (the unreduced sets, for comparison)."""
    if a in ps: return False
    if not reduce:
        ps.append(a)
        return False
    red = any(u > a and paths_meet(mvs[u], mvs[a]) for u in ps)
    ps[:] = [u for u in ps if not (u < a and paths_meet(mvs[u], mvs[a]))]
    if red: return False
    if len(ps) == 8: return True
    ps.append(a)
    return False


def graph(shape, moves, goff, reduce=True):
    """Transliteration of graph_core (rr_batch_graph.hpp), threads run one after the other.
    reduce=False keeps every distinct in-group previous toucher (no pred_add reduction, no limit)."""
    W, H = shape[0], shape[1]
    K = len(moves); G = len(goff) - 1; WH = W * H
    mvs = [tuple(int(v) for v in m) for m in moves]
    def trap(m, s):
        sx, sy, dx, dy = m
        hx = abs(dx - sx)
        if s <= hx: return sy * W + (sx + s if dx >= sx else sx - s)
        v = s - hx
        return (sy + v if dy >= sy else sy - v) * W + dx
    L = lambda m: abs(m[2] - m[0]) + abs(m[3] - m[1])
    grp = [0] * K
    for g in range(G):
        for b in range(goff[g], goff[g + 1]): grp[b] = g
    cell = [0] * (WH + 1)
    for b in range(K):
        for s in range(L(mvs[b]) + 1): cell[trap(mvs[b], s)] += 1
    run = 0
    for c in range(WH + 1):
        v = cell[c] if c < WH else 0
        cell[c] = run; run += v
    touch = [None] * (cell[WH])
    # scatter in an arbitrary thread order (reverse) to mimic atomics
    for b in reversed(range(K)):
        for s in range(L(mvs[b]) + 1):
            c = trap(mvs[b], s); touch[cell[c]] = b; cell[c] += 1
    for c in range(WH):
        lo = cell[c - 1] if c else 0
        touch[lo:cell[c]] = sorted(touch[lo:cell[c]])
    pend = [0] * K; preds = [[] for _ in range(K)]; soff = [0] * (K + 1); gbits = {}
    ovf = False
    for b in range(K):
        g = grp[b]; ps = []; gs = []; last = None
        for s in range(L(mvs[b]) + 1):
            c = trap(mvs[b], s)
            lo = cell[c - 1] if c else 0; hi = cell[c]
            if touch[lo] == b: continue
            while hi - lo > 1:
                mid = (lo + hi) >> 1
                if touch[mid] < b: lo = mid
                else: hi = mid
            a = touch[lo]
            if a == last: continue
            last = a
            if grp[a] == g:
                ovf |= pred_add(ps, a, mvs, reduce)
            else:
                if grp[a] not in gs: gs.append(grp[a])
        pend[b] = len(ps); preds[b] = ps
        for a in ps: soff[a] += 1
        for x in gs: gbits.setdefault(g, set()).add(x)
    assert not ovf
    run = 0
    for a in range(K + 1):
        v = soff[a] if a < K else 0
        soff[a] = run; run += v
    slist = [None] * soff[K]; fill = [0] * K
    for b in reversed(range(K)):
        for a in preds[b]:
            slist[soff[a] + fill[a]] = b; fill[a] += 1
    nx = []; extra = 0
    for a in range(K):
        lo, ns = soff[a], soff[a + 1] - soff[a]
        code = 0
        if ns == 1:
            n = slist[lo]
            code = ((1 << 14) | (n - a)) if (pend[n] == 1 and n - a <= 16383) else (2 << 14)
        elif ns > 1:
            code = 2 << 14; extra += ns - 1
        nx.append(code)
    heads = [[b for b in range(goff[g], goff[g + 1]) if pend[b] == 0] for g in range(G)]
    gpend = [len(gbits.get(g, ())) for g in range(G)]
    gw = [[h for h in range(G) if g in gbits.get(h, ())] for g in range(G)]
    succ = [slist[soff[a]:soff[a + 1]] for a in range(K)]
    mv = [m[0] | (m[1] << 8) | (m[2] << 16) | (m[3] << 24) for m in mvs]
    HN = sum(len(h) for h in heads)
    return dict(K=K, G=G, mv=mv, nx=nx, succ=succ, pend=pend, gw=gw, gpend=gpend, heads=heads,
                bound=HN + extra, goff=list(goff))


def walk_rows(W, m, y0, y1):
    """Traps of move m = (sx, sy, dx, dy) in rows [y0, y1), as walk_rows (rr_batch_graph.hpp)."""
    sx, sy, dx, dy = m
    out = []
    if y0 <= sy < y1:
        st = 1 if dx >= sx else -1
        out += [sy * W + sx + st * s for s in range(abs(dx - sx) + 1)]
    vy = abs(dy - sy)
    if vy:
        if dy > sy: lo, hi = max(1, y0 - sy), min(vy, y1 - 1 - sy)
        else: lo, hi = max(1, sy - y1 + 1), min(vy, sy - y0)
        st = 1 if dy > sy else -1
        out += [(sy + st * v) * W + dx for v in range(lo, hi + 1)]
    return out


def graph_tiled(shape, moves, goff, tile_bytes, reduce=True):
    """The tiled build (graph_tiled, rr_batch_graph.hpp) step by step: row counts through a
    difference array, greedy row ranges of at most 64 rows whose cells (4 B + 4) and visits (2 B)
    fit tile_bytes, per-range move lists, then per range the touch lists and previous touchers
    (the kernel scans each unsorted list for the largest index below the walking move; the model
    sorts and takes the maximum below, the same previous toucher).
    Returns (in-group predecessor sets, group predecessor sets, ranges) or None when a single row
    does not fit."""
    W, H = shape[0], shape[1]
    mvs = [tuple(int(v) for v in m) for m in moves]
    K = len(mvs); G = len(goff) - 1
    grp = [0] * K
    for g in range(G):
        for b in range(goff[g], goff[g + 1]): grp[b] = g
    rowc = [0] * (H + 1)
    for (sx, sy, dx, dy) in mvs:
        nh = abs(dx - sx) + 1
        rowc[sy] += nh; rowc[sy + 1] -= nh
        if dy != sy:
            vlo, vhi = (sy + 1, dy) if dy > sy else (dy, sy - 1)
            rowc[vlo] += 1; rowc[vhi + 1] -= 1
    cum, run, acc = [0] * H, 0, 0
    for y in range(H):
        acc += rowc[y]; run += acc; cum[y] = run
    rs, rrow, y0, before = [], [0] * H, 0, 0
    while y0 < H:
        n = 0
        for lane in range(64):
            y1 = y0 + 1 + lane
            if y1 <= H and 4 * ((y1 - y0) * W + 1) + 2 * (cum[y1 - 1] - before) <= tile_bytes: n += 1
        if n == 0: return None
        for y in range(y0, y0 + n): rrow[y] = len(rs)
        rs.append(y0); before = cum[y0 + n - 1]; y0 += n
    rs.append(H); R = len(rs) - 1
    lists = [[] for _ in range(R)]
    for b, (sx, sy, dx, dy) in enumerate(mvs):
        for r in range(rrow[min(sy, dy)], rrow[max(sy, dy)] + 1): lists[r].append(b)
    assert sum(len(l) for l in lists) <= K + sum(abs(m[2] - m[0]) + abs(m[3] - m[1]) for m in mvs)
    preds = [[] for _ in range(K)]; gbits = {}; ovf = False
    for r in range(R):
        y0, y1 = rs[r], rs[r + 1]; c0, nc = y0 * W, (y1 - y0) * W
        touch = {}
        for b in reversed(lists[r]):            # arbitrary arrival order
            w = walk_rows(W, mvs[b], y0, y1)
            assert w, "a listed move has no trap in the range"
            for c in w:
                assert c0 <= c < c0 + nc
                touch.setdefault(c, []).append(b)
        visits = sum(len(v) for v in touch.values())
        assert visits == cum[y1 - 1] - (cum[y0 - 1] if y0 else 0)
        assert 4 * (nc + 1) + 2 * visits <= tile_bytes
        for c in touch: touch[c].sort()
        for b in lists[r]:
            g, glo = grp[b], goff[grp[b]]
            last = lastg = None
            for c in walk_rows(W, mvs[b], y0, y1):
                L = touch[c]
                if L[0] == b: continue
                a = max(v for v in L if v < b)
                if a == last: continue
                last = a
                if a >= glo:
                    ovf |= pred_add(preds[b], a, mvs, reduce)
                elif grp[a] != lastg:
                    lastg = grp[a]
                    gbits.setdefault(g, set()).add(grp[a])
    assert not ovf
    return [set(p) for p in preds], gbits, R


def wide_graph(shape, moves, goff):
    """The wide path's graph build (rr_batch_wide.hip, graph): groups in order; a move's in-group
    predecessors are the earlier moves of its group whose paths meet its own, scanned from the
    nearest down and skipped when they meet a member already kept (at most 8); a group's
    predecessor groups are the last groups to touch each of its traps before it (a per-trap
    word, stamped by each group after it has read).  Returns the graph in the form loop() takes
    (release codes, successor lists, group lists, heads)."""
    W, H = shape[0], shape[1]
    mvs = [tuple(int(v) for v in m) for m in moves]
    K = len(mvs); G = len(goff) - 1
    lastg = [None] * (W * H)
    preds = [[] for _ in range(K)]
    gpred = [set() for _ in range(G)]

    def traps(m):
        sx, sy, dx, dy = m
        st = 1 if dx >= sx else -1
        out = [sy * W + x for x in range(sx, dx + st, st)]
        st = 1 if dy >= sy else -1
        return out + [y * W + dx for y in range(sy + st, dy + st, st)]

    goff = [int(v) for v in goff]
    for h in range(G):
        lo, hi = goff[h], goff[h + 1]
        for b in range(lo, hi):
            ps = []
            for a in range(b - 1, lo - 1, -1):
                if not paths_meet(mvs[a], mvs[b]): continue
                if any(paths_meet(mvs[u], mvs[a]) for u in ps): continue
                assert len(ps) < 8, "in-group predecessor set overflow"
                ps.append(a)
            preds[b] = ps
        for b in range(lo, hi):
            for c in traps(mvs[b]):
                if lastg[c] is not None: gpred[h].add(lastg[c])
        for b in range(lo, hi):
            for c in traps(mvs[b]): lastg[c] = h
    pend = [len(p) for p in preds]
    succ = [[] for _ in range(K)]
    for b in range(K):
        for a in preds[b]: succ[a].append(b)
    nx = []; extra = 0
    for a in range(K):
        ns = len(succ[a]); code = 0
        if ns == 1:
            n = succ[a][0]
            code = ((1 << 14) | (n - a)) if (pend[n] == 1 and n - a <= 16383) else (2 << 14)
        elif ns > 1:
            code = 2 << 14; extra += ns - 1
        nx.append(code)
    heads = [[b for b in range(goff[g], goff[g + 1]) if pend[b] == 0] for g in range(G)]
    gw = [sorted(h for h in range(G) if g in gpred[h]) for g in range(G)]
    mv = [m[0] | (m[1] << 8) | (m[2] << 16) | (m[3] << 24) for m in mvs]
    return dict(K=K, G=G, mv=mv, nx=nx, succ=succ, pend=pend, gw=gw, gpend=[len(x) for x in gpred], heads=heads,
                bound=sum(len(x) for x in heads) + extra, goff=list(goff), preds=preds)
