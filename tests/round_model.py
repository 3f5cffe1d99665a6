"""A plain CPU model of one multi-pick round of the sampler (test support).

The GPU sampler settles many selections per exchange (`csrc/sample_rounds.hip`):
every workgroup runs R steps of local FPS on its own points (lookahead),
publishes its candidates, their local distances and runner-ups and its
bound, and every workgroup replays the same merge, which certifies
candidates in key order.  This module writes that round out in numpy with
groups of points instead of workgroups and tiles (pruning never changes a
distance, so it is left out), with the merge taken step by step as the
kernel does it:

  - list the candidates above S* (the largest bound), cut at a key boundary
    when there are more than `klist`;
  - for every listed candidate, its rank in key order and the set of listed
    candidates with a larger key whose distance to it is below its listed
    distance (the ones that would lower it);
  - walk: a live candidate fails when a live member of its set exists; the
    first failure is the failing candidate with the largest key; the live
    candidates above it are picks and stay live; the failed one gets its
    true distance, the bound rises to its runner-up, its group's later
    candidates and every key at or below the bound leave the list, it goes
    back in if its new key is above the bound, and the walk goes on;
  - order the picks by current key with the list ranks corrected for the
    candidates whose keys changed or that left the list.

It shares no code with the HIP path and none with the oracle; tests run it
against the oracle (Algorithm 1 with the Sec. 3.1 tie rule), so a mistake in
the certification rule shows up as a different sequence without a GPU.
"""
import numpy as np

f32 = np.float32
MAX_FAIL = 64


def d2(p, s):
    """FP32 squared distance ((dx*dx + dy*dy) + dz*dz), dx = fl(p_x - s_x)."""
    dx = (p[..., 0] - s[0]).astype(f32)
    dy = (p[..., 1] - s[1]).astype(f32)
    dz = (p[..., 2] - s[2]).astype(f32)
    return ((dx * dx).astype(f32) + (dy * dy).astype(f32)).astype(f32) + (dz * dz).astype(f32)


def fbits(x):
    return int(np.float32(x).view(np.uint32))


def key(d, o):
    """(distance bits, ~original index): the larger key is the FPS choice."""
    return (fbits(d) << 32) | ((~int(o)) & 0xffffffff)


def run(P, m, start, G, R, klist=128, bound="runner"):
    """FPS of m points from start with G groups of R candidates per round.
    A group's bound is the runner-up of its last step (bound="runner"), or
    the largest local key after all R steps (bound="next").
    Returns (indices, distances, rounds, failures)."""
    n = len(P)
    groups = [np.arange(g, n, G) for g in range(G)]
    D = d2(P, P[start]).astype(f32)
    out, outd = [start], [np.float32(np.inf)]
    j, rounds, fails_total = 1, 0, 0
    while j < m:
        rounds += 1
        # lookahead: R local FPS steps per group on a private copy
        cands, bounds = {}, {}
        for g in range(G):
            idx = groups[g]
            if len(idx) == 0:
                bounds[g] = 0
                continue
            Dl = D[idx].copy()
            for s in range(R + 1):
                keys = [key(Dl[t], idx[t]) for t in range(len(idx))]
                kmax = max(keys)
                if s == R or kmax == 0:
                    bounds[g] = kmax
                    break
                t = keys.index(kmax)
                others = keys[:t] + keys[t + 1:]
                runner = max(others) if others else 0
                cands[g * R + s] = (idx[t], Dl[t], runner >> 32)
                if bound == "runner" and s == R - 1:
                    # applying l_R only lowers the other points' keys, and
                    # its own becomes (0, its index)
                    bounds[g] = max(runner, key(0.0, idx[t]))
                    break
                dd = d2(P[idx], P[idx[t]])
                Dl = np.where(dd < Dl, dd, Dl).astype(f32)
        bkey = {c: (key(cands[c][1], cands[c][0]) if c in cands else 0) for c in range(G * R)}
        smax = max(bounds.values())
        lst = [c for c in range(G * R)
               if bkey[c] != 0 and (bkey[c] > smax or (bkey[c] == smax and bounds[c // R] == smax))]
        scur = smax
        if len(lst) > klist:
            srt = sorted(lst, key=lambda c: (-bkey[c], lst.index(c)))
            W = klist
            while W > 1 and bkey[srt[W - 1]] == bkey[srt[W]]:
                W -= 1
            scur = max(scur, bkey[srt[W]])
            lst = srt[:W]
        W = len(lst)
        pmax = min(W, m - j)
        kc = [bkey[c] for c in lst]
        xyz = [P[cands[c][0]] for c in lst]
        ld = [f32(cands[c][1]) for c in lst]
        rank = [sum(1 for q in range(W) if kc[q] > kc[i] or (kc[q] == kc[i] and q < i)) for i in range(W)]
        sets = [{q for q in range(W) if kc[q] > kc[i] and d2(xyz[i][None], xyz[q])[0] < ld[i]} for i in range(W)]
        live, X, relisted, nfail = set(range(W)), set(), set(), 0
        dist = {c: f32(cands[c][1]) for c in lst}
        while True:
            failing = [i for i in live if sets[i] & live]
            if not failing:
                npick = min(len(live), pmax)
                break
            kf = max(kc[i] for i in failing)
            fi = next(i for i in failing if kc[i] == kf)
            picks = {q for q in live if kc[q] > kf}
            npick = len(picks)
            if npick >= pmax:
                npick = pmax
                break
            nfail += 1
            if nfail > MAX_FAIL:
                break
            c = lst[fi]
            tv = min([np.float32(np.inf)] + [d2(xyz[fi][None], xyz[q])[0] for q in sets[fi] & live])
            tf = f32(min(tv, np.uint32(kf >> 32).view(np.float32)))
            kt = (fbits(tf) << 32) | (kf & 0xffffffff)
            scur = max(scur, (int(cands[c][2]) << 32) | 0xffffffff)
            later = {q for q in live if lst[q] // R == c // R and lst[q] % R > c % R} - picks
            X |= later
            live -= later
            live -= {q for q in live if kc[q] <= scur} - picks
            if kt > scur:
                live.add(fi)
            else:
                live.discard(fi)
            X.add(fi)
            relisted.add(fi)
            kc[fi] = kt
            for i in range(W):
                if kc[i] > kt:
                    sets[i].discard(fi)
            sets[fi] = {q for q in range(W) if kc[q] > kt and d2(xyz[fi][None], xyz[q])[0] < tf}
            dist[c] = tf
        order = list(rank)
        for q in X:
            up = q in relisted and q in live
            for i in range(W):
                order[i] += (1 if (up and kc[q] > kc[i]) else 0) - (1 if rank[q] < rank[i] else 0)
        for q in relisted & live:
            order[q] = sum(1 for i in live if kc[i] > kc[q])
        chosen = [None] * npick
        for i in live:
            if order[i] < npick:
                assert chosen[order[i]] is None, "two picks share a position"
                chosen[order[i]] = i
        assert npick > 0 and all(x is not None for x in chosen), "a round settled nothing or left a hole"
        fails_total += nfail
        for i in chosen:
            c = lst[i]
            pt = cands[c][0]
            out.append(pt)
            outd.append(dist[c])
            dd = d2(P, P[pt])
            D = np.where(dd < D, dd, D).astype(f32)
        j += npick
    return np.array(out[:m]), np.array(outd[:m], dtype=f32), rounds, fails_total
