"""Dynamic regrid of the oracle (test infrastructure).

The paper refines statically and names dynamic refinement as future work
(section 6); the regrid applied here uses the paper's own inter-level
operators on the state between coarse steps (the post-streaming state of
Algorithm 1):

* a leaf flagged for refinement is split and each new fine cell takes all 19
  PDFs of the coarse cell containing it (eq. ctof);
* 8 sibling leaves all flagged for coarsening merge and each new coarse cell
  takes the mean of its 8 children (eq. ftoc);
* leaves split only by the 2:1 balance are exploded in the same way.

Leaf-set rules: split flagged leaves (below max_level), restore the 2:1
balance by splitting, then merge sibling groups level by level from the
finest down, a merge being kept only if no leaf two or more levels finer
than the merged parent touches it (checked here by brute force over all
leaves, with closed boxes on the periodic domain).
"""

from __future__ import annotations

import numpy as np

from .forest import Forest


def _children(leaf):
    L, x, y, z = leaf
    return [(L + 1, 2 * x + ox, 2 * y + oy, 2 * z + oz) for oz in (0, 1) for oy in (0, 1) for ox in (0, 1)]


def _touches(a, b, R, Lm):
    """Closed boxes of leaves a and b meet on the periodic domain."""
    for axis in range(3):
        D = R[axis] << Lm
        sa, sb = 1 << (Lm - a[0]), 1 << (Lm - b[0])
        a0, a1 = a[axis + 1] * sa, (a[axis + 1] + 1) * sa
        b0, b1 = b[axis + 1] * sb, (b[axis + 1] + 1) * sb
        if not any(b0 + k <= a1 and a0 <= b1 + k for k in (-D, 0, D)):
            return False
    return True


def regrid_forest(forest: Forest, flags, max_level: int) -> Forest:
    leaves = forest.canonical_leaves()
    if len(flags) != len(leaves):
        raise ValueError("one flag per leaf expected")
    new = set(forest.leaves)
    coarsen = set()
    for leaf, fl in zip(leaves, flags):
        if fl > 0 and leaf[0] < max_level:
            new.remove(leaf)
            new.update(_children(leaf))
        elif fl < 0 and leaf[0] > 0:
            coarsen.add(leaf)
    f2 = Forest(forest.R, forest.n, new, forest.periodic)
    f2.balance()
    Lm = max(leaf[0] for leaf in f2.leaves) + 1
    for L in range(max(leaf[0] for leaf in f2.leaves), 0, -1):
        parents = sorted({(L - 1, x >> 1, y >> 1, z >> 1) for (l, x, y, z) in coarsen if l == L})
        for P in parents:
            kids = _children(P)
            if not all(k in coarsen and k in f2.leaves for k in kids):
                continue
            if any(q[0] > L and _touches(P, q, f2.R, Lm) for q in f2.leaves):
                continue
            for k in kids:
                f2.leaves.remove(k)
            f2.leaves.add(P)
    f2.max_level = max(leaf[0] for leaf in f2.leaves)
    f2.check_cover()
    assert f2.is_balanced()
    return f2


def remap_interior(old_forest: Forest, old_pdfs, new_forest: Forest):
    """Interior PDFs of the new forest from those of the old one.

    old_pdfs: list over levels of (N_L, 19) arrays in canonical cell order.
    Returns the same structure for the new forest."""
    n = old_forest.n
    loc = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
    loc = loc.transpose(2, 1, 0, 3).reshape(-1, 3)  # x fastest
    old_index = {}
    for L in range(old_forest.max_level + 1):
        for b, pos in enumerate(old_forest.level_blocks(L)):
            old_index[(L,) + tuple(int(v) for v in pos)] = b
    out = []
    for L in range(new_forest.max_level + 1):
        blocks = new_forest.level_blocks(L)
        F = np.empty((len(blocks) * n ** 3, 19))
        for b, pos in enumerate(blocks):
            key = (L,) + tuple(int(v) for v in pos)
            dst = F[b * n ** 3:(b + 1) * n ** 3]
            if key in old_index:
                ob = old_index[key]
                dst[:] = old_pdfs[L][ob * n ** 3:(ob + 1) * n ** 3]
                continue
            anc = None
            for up in range(1, L + 1):
                cand = (L - up,) + tuple(int(v) >> up for v in pos)
                if cand in old_index:
                    anc = (up, cand)
                    break
            if anc is not None:
                up, cand = anc
                g = pos[None, :] * n + loc                      # global cells of the new block
                og = g >> up                                     # cell of the old ancestor level
                ol = og - np.array(cand[1:]) * n                 # local inside the old block
                idx = old_index[cand] * n ** 3 + ol[:, 0] + n * (ol[:, 1] + n * ol[:, 2])
                dst[:] = old_pdfs[L - up][idx]
                continue
            # the 8 children are old leaves: mean over them
            acc = np.zeros_like(dst)
            g = pos[None, :] * n + loc
            for oz in (0, 1):
                for oy in (0, 1):
                    for ox in (0, 1):
                        c = 2 * g + np.array([ox, oy, oz])
                        cb = c // n
                        idx = np.empty(len(c), dtype=np.int64)
                        for i in range(len(c)):
                            idx[i] = old_index[(L + 1,) + tuple(int(v) for v in cb[i])] * n ** 3 + \
                                int(c[i, 0] % n) + n * (int(c[i, 1] % n) + n * int(c[i, 2] % n))
                        acc += old_pdfs[L + 1][idx]
            dst[:] = acc / 8.0
        out.append(F)
    return out
