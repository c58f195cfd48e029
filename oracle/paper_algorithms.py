"""The paper's four Hierarchy-Scan algorithms in FP64 NumPy -- TEST INFRASTRUCTURE.

Each routine takes one character's parent array (``-1`` = root, parents
before children) and its local 4x4 matrices, and returns the global
matrices.  They are written from the algorithm descriptions under the
readings stated below and exist to pin those readings: every one must agree
with the sequential definition (``oracle.scan_matrices``) to rounding.  All
rounds are synchronous: every joint reads the values of the previous round
(the in-place updates of the printed pseudo-code would otherwise race).

Readings (the printed pseudo-code has slips):

* Algorithm 1 (Sec. 2, Gateau's per-joint walk): the loop advances the walker
  to the parent of the *current* ancestor, multiplying the ancestors' local
  matrices on the left.
* Algorithm 2 (Sec. 3.1, Eq. 2): round d combines each joint with its
  2^(d-1)-th ancestor of the previous round (Wyllie pointer jumping);
  ceil(log2 depth) rounds suffice.
* Algorithm 3 (Sec. 3.2.1): blocks of 64 consecutive ids; the in-block rounds
  only follow ancestors inside the block; then each joint walks
  MaxParentOutBlock, multiplying the in-block partial product of each
  out-of-block ancestor it reaches.
* Algorithm 4 (Sec. 3.2.2): in-block, seven single-parent steps give an
  8-node window, then seven hops of stride 8 over those windows give the
  64-node block partial; then the MaxParentOutBlock walk of Algorithm 3.
"""
import math

import numpy as np


def depth_levels(parents):
    """Depth of each joint in levels, the root being level 1."""
    lev = np.zeros(len(parents), np.int64)
    for j, p in enumerate(parents):
        lev[j] = 1 if p < 0 else lev[p] + 1
    return lev


def alg1_walk_to_root(parents, local):
    """Algorithm 1: every joint multiplies in all of its ancestors' local matrices."""
    n = len(parents)
    out = np.empty_like(local)
    for j in range(n):
        m = local[j].copy()
        cur = parents[j]
        while cur >= 0:
            m = local[cur] @ m
            cur = parents[cur]
        out[j] = m
    return out


def alg2_pointer_jumping(parents, local, rounds=None):
    """Algorithm 2: synchronous pointer jumping over all joints."""
    n = len(parents)
    m = local.copy()
    anc = np.asarray(parents, np.int64).copy()
    if rounds is None:
        d = int(depth_levels(parents).max()) if n else 0
        rounds = math.ceil(math.log2(d)) if d > 1 else 0
    for _ in range(rounds):
        new_m = m.copy()
        new_anc = anc.copy()
        for j in range(n):
            a = anc[j]
            if a >= 0:
                new_m[j] = m[a] @ m[j]
                new_anc[j] = anc[a]
        m, anc = new_m, new_anc
    return m


def _block_of(j, block):
    return j // block


def max_parent_out_block(parents, block=64):
    """For each joint, its nearest ancestor outside its own block (-1 if none).

    Ids grow along every root-to-leaf path, so the in-block part of a path is
    contiguous; this is the parent of the topmost in-block ancestor.
    """
    n = len(parents)
    out = np.full(n, -1, np.int64)
    for j in range(n):
        cur = parents[j]
        while cur >= 0 and _block_of(cur, block) == _block_of(j, block):
            cur = parents[cur]
        out[j] = cur
    return out


def _walk_out_of_block(parents, partial, block):
    """Cross-block phase shared by Algorithms 3 and 4 (on a snapshot)."""
    mpob = max_parent_out_block(parents, block)
    out = partial.copy()
    for j in range(len(parents)):
        cur = mpob[j]
        while cur >= 0:
            out[j] = partial[cur] @ out[j]
            cur = mpob[cur]
    return out


def alg3_blocks(parents, local, block=64):
    """Algorithm 3: in-block pointer jumping (log2(block) rounds), then the walk."""
    n = len(parents)
    inb = np.array([p if p >= 0 and _block_of(p, block) == _block_of(j, block) else -1
                    for j, p in enumerate(parents)], np.int64)
    m = local.copy()
    anc = inb.copy()
    for _ in range(int(math.log2(block))):
        new_m = m.copy()
        new_anc = anc.copy()
        for j in range(n):
            a = anc[j]
            if a >= 0:
                new_m[j] = m[a] @ m[j]
                new_anc[j] = anc[a]
        m, anc = new_m, new_anc
    return _walk_out_of_block(parents, m, block)


def alg4_state_compression(parents, local, block=64, window=8):
    """Algorithm 4: 7 single steps (window of 8), 7 hops of 8, then the walk."""
    n = len(parents)
    inb = [p if p >= 0 and _block_of(p, block) == _block_of(j, block) else -1
           for j, p in enumerate(parents)]

    def up(j, k):
        for _ in range(k):
            if j < 0:
                return -1
            j = inb[j]
        return j

    # phase 1: window W_j = product of the local matrices of j and up to
    # window-1 in-block ancestors (reads the untouched local matrices).
    win = local.copy()
    for j in range(n):
        cur = inb[j]
        for _ in range(window - 1):
            if cur < 0:
                break
            win[j] = local[cur] @ win[j]
            cur = inb[cur]
    # phase 2: hops of stride `window` over the phase-1 windows (snapshot).
    part = win.copy()
    hops = block // window - 1
    for j in range(n):
        cur = up(j, window)
        for _ in range(hops):
            if cur < 0:
                break
            part[j] = win[cur] @ part[j]
            cur = up(cur, window)
    return _walk_out_of_block(parents, part, block)
