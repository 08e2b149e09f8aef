"""Oracle: compressed sparse fiber (CSF) packing.  TEST INFRASTRUCTURE ONLY.

CSF stores a sigma-sorted tensor as a tree whose levels follow sigma: level d
holds the indices of mode sigma_d, each node's children are the next mode's
indices under it, and the leaves are the nonzeros (Sec. 1, Sec. 2, Sec. 2.2).
The paper fixes no array layout; the one used here compresses every level:

* F_0 = 1 (the root).  For 1 <= d < r a level-d fiber is a maximal run of
  consecutive nonzeros that share (sigma_1..sigma_d); at d = r every nonzero is
  its own leaf, so duplicated coordinates stay separate leaves (merging them
  would need arithmetic on values).
* crd[d-1] has F_d entries: the sigma_d coordinate of each level-d fiber.
* pos[d-1] has F_{d-1} + 1 entries: the children of level-(d-1) fiber p are the
  level-d fibers pos[d-1][p] .. pos[d-1][p+1] - 1.

Pure Python loops; meant for small inputs.
"""


def pack_csf(crd, sigma):
    """crd: r coordinate sequences already sorted under sigma.  Returns (pos, crd_levels)."""
    r = len(sigma)
    n = len(crd[0]) if r else 0
    pos, levels = [], []
    parent_starts = [j == 0 for j in range(n)]  # the root's only "fiber" starts at 0
    for d in range(1, r + 1):
        head = sigma[:d]
        starts = []
        for j in range(n):
            if d == r or j == 0:
                starts.append(True)
            else:
                starts.append(any(crd[m][j] != crd[m][j - 1] for m in head))
        levels.append([int(crd[sigma[d - 1]][j]) for j in range(n) if starts[j]])
        p, f = [], 0
        for j in range(n):
            if parent_starts[j]:
                p.append(f)  # children of the parent fiber beginning at j start at fiber f
            if starts[j]:
                f += 1
        if d == 1:
            p = [0]  # one root, whatever n is
        p.append(f)
        pos.append(p)
        parent_starts = starts
    return pos, levels


def unpack_csf(pos, levels, sigma):
    """Walk the tree depth-first and list every leaf's coordinate tuple, in
    the mode order of the original tensor (the inverse of pack_csf)."""
    r = len(sigma)
    out = [[] for _ in range(r)]

    def walk(d, p, path):
        # children of fiber p at level d-1 live at level d
        for f in range(pos[d - 1][p], pos[d - 1][p + 1]):
            here = path + [levels[d - 1][f]]
            if d == r:
                for m_i, m in enumerate(sigma):
                    out[m].append(here[m_i])
            else:
                walk(d + 1, f, here)

    if r:
        walk(1, 0, [])
    return out
