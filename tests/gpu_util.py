"""Helpers shared by the GPU tests (CPU-side reference replays)."""
import numpy as np

from oracle import nystrom


def replay_alg1_E(pts, a, fac, n_boxes_levels):
    """Algorithm 1's E_i = (R F^{-1} R^T)^{-1} computed on the CPU for every
    non-root box, in the library's point ordering and with the library's T
    matrices (read back), so that the comparison isolates the elimination
    arithmetic.  Returns {box: E}."""
    E = {}
    act = {}
    info = {}
    nb = fac.stats()["n_boxes"]
    for b in range(nb):
        info[b] = fac.box_info(b)
        act[b] = fac.block(b, 2)
    children = {}
    for b in range(nb):
        p = info[b]["parent"]
        if p >= 0:
            children.setdefault(p, []).append(b)
    root = nb - 1
    for b in range(nb - 1):
        k, r = info[b]["k"], info[b]["r"]
        ids = act[b]
        if b not in children:
            F = nystrom.assemble(pts, a, rows=ids, cols=ids)
        else:
            c1, c2 = children[b]
            F = nystrom.assemble(pts, a, rows=ids, cols=ids)
            # replace the diagonal child blocks by the children's E (Alg. 1, line 5)
            for c in (c1, c2):
                kc = info[c]["k"]
                sk = act[c][:kc]
                pos = np.array([np.nonzero(ids == g)[0][0] for g in sk])
                F[np.ix_(pos, pos)] = E[c]
        if r:
            T = fac.block(b, 0)
            R = np.hstack([np.eye(k), T])
            E[b] = np.linalg.inv(R @ np.linalg.inv(F) @ R.T)
        else:
            E[b] = F
    return E
