"""The ordering rules of the level-scheduled kernels, as a model run under random
interleavings (CPU).  The factorization and the triangular sweeps order their dependency
levels without barriers: each wavefront publishes a progress level (every row of it below
that level is finished), a unit of work of level or phase p waits until the minimum over the
wavefronts reaches p, and a wavefront raises its level after finishing a row.  The sweeps
also reuse LDS slots: a row's slot is free from one level after its last reader on.

On random lower-triangular dependency patterns (levels from the pattern, rows dealt
round-robin in level order, leading tasks of split rows at one phase past their latest
input), every interleaving drawn must finish (no state where work remains and nothing can
run), every read must follow the write it needs, and no slot may be overwritten before its
last reader has read it.
"""
import numpy as np
import pytest


def random_pattern(rng, n, band, density):
    """cols[i]: the rows i depends on (all < i), within a band, as RCM orderings give."""
    cols = []
    for i in range(n):
        lo = max(0, i - band)
        c = [j for j in range(lo, i) if rng.random() < density]
        if i > 0 and rng.random() < 0.8:
            c.append(i - 1)  # the chain RCM leaves: about one row per level
        cols.append(sorted(set(c)))
    return cols


def levels_of(cols):
    lv = []
    for c in cols:
        lv.append(1 + max((lv[j] for j in c), default=-1))
    return lv


def colour_slots(cols, lv):
    """Slots live from a row's level to its last reader's level; freed one level later."""
    n = len(cols)
    last = [-1] * n
    for i, c in enumerate(cols):
        for j in c:
            last[j] = max(last[j], lv[i])
    nl = max(lv) + 1
    release = [[] for _ in range(nl + 1)]
    free, used, slot = [], 0, [-1] * n
    order = sorted(range(n), key=lambda i: (lv[i], i))
    for L in range(nl):
        free += release[L]
        for i in (i for i in order if lv[i] == L):
            if last[i] < 0:
                continue
            if free:
                slot[i] = free.pop()
            else:
                slot[i] = used
                used += 1
            release[last[i] + 1].append(slot[i])
    return slot, last


def sweep_tasks(cols, lv, nw, mb):
    """Per wavefront: tasks (row, blocks, phase, final) in schedule order."""
    order = sorted(range(len(cols)), key=lambda i: (lv[i], i))
    waves = [[] for _ in range(nw)]
    for q, i in enumerate(order):
        c = cols[i]
        chunks = [c[k:k + mb] for k in range(0, len(c), mb)] or [[]]
        for k, ch in enumerate(chunks):
            final = k == len(chunks) - 1
            ph = lv[i] if final else 1 + max(lv[j] for j in ch)
            waves[q % nw].append((i, ch, ph, final))
    return waves


def run_sweep(rng, cols, lv, nw, mb, early=0):
    """early > 0 lets every task start that many phases too soon (a broken rule)."""
    slot, last = colour_slots(cols, lv)
    waves = [[(i, ch, max(0, ph - early), f) for (i, ch, ph, f) in w] for w in sweep_tasks(cols, lv, nw, mb)]
    nl = max(lv) + 1
    pos = [0] * nw
    # a wavefront's published phase: the row phase of its next task (nl when done)
    prog = [lv[w[0][0]] if w else nl for w in waves]
    done = [False] * len(cols)
    holder = {}      # slot -> row whose value it holds
    reads_left = {}  # row -> readers not yet finished
    for i, c in enumerate(cols):
        for j in c:
            reads_left[j] = reads_left.get(j, 0) + 1
    while True:
        ready = [w for w in range(nw) if pos[w] < len(waves[w]) and min(prog) >= waves[w][pos[w]][2]]
        if not ready:
            assert all(pos[w] == len(waves[w]) for w in range(nw)), "deadlock"
            return
        w = ready[rng.integers(len(ready))]
        i, ch, ph, final = waves[w][pos[w]]
        for j in ch:  # reads: the column row is finished and its slot still holds it
            assert done[j], f"row {i} read row {j} before it was written"
            assert holder.get(slot[j]) == j, f"slot of row {j} overwritten before row {i} read it"
        if final:
            # the readers of this row's columns are counted when the row finishes
            for j in cols[i]:
                reads_left[j] -= 1
            if slot[i] >= 0:
                prev = holder.get(slot[i])
                assert prev is None or reads_left.get(prev, 0) == 0, \
                    f"row {i} overwrote the slot of row {prev} with readers left"
                holder[slot[i]] = i
            done[i] = True
        pos[w] += 1
        nxt = lv[waves[w][pos[w]][0]] if pos[w] < len(waves[w]) else nl
        if nxt > prog[w]:
            prog[w] = nxt


def run_factor(rng, cols, lv, nw):
    """Rows round-robin in level order; a row's pivot groups in ascending pivot order, each
    waiting until min over wavefronts of the progress level exceeds the pivot's level."""
    order = sorted(range(len(cols)), key=lambda i: (lv[i], i))
    waves = [[] for _ in range(nw)]
    for q, i in enumerate(order):
        waves[q % nw].append(i)
    nl = max(lv) + 1
    prog = [lv[w[0]] if w else nl for w in waves]
    row_pos, grp_pos = [0] * nw, [0] * nw
    final = [False] * len(cols)
    while True:
        ready = []
        for w in range(nw):
            if row_pos[w] == len(waves[w]):
                continue
            i = waves[w][row_pos[w]]
            g = grp_pos[w]
            if g == len(cols[i]) or min(prog) > lv[cols[i][g]]:
                ready.append(w)
        if not ready:
            assert all(row_pos[w] == len(waves[w]) for w in range(nw)), "deadlock"
            return
        w = ready[rng.integers(len(ready))]
        i = waves[w][row_pos[w]]
        g = grp_pos[w]
        if g < len(cols[i]):
            assert final[cols[i][g]], f"row {i} used pivot {cols[i][g]} before it was final"
            grp_pos[w] += 1
            continue
        final[i] = True  # inverse and write-back done, then the release
        row_pos[w] += 1
        grp_pos[w] = 0
        nxt = lv[waves[w][row_pos[w]]] if row_pos[w] < len(waves[w]) else nl
        if nxt > prog[w]:
            prog[w] = nxt


@pytest.mark.parametrize("seed", range(6))
def test_sweep_waits_and_slot_reuse(seed):
    rng = np.random.default_rng(seed)
    for trial in range(20):
        n = int(rng.integers(20, 120))
        cols = random_pattern(rng, n, band=int(rng.integers(3, 25)), density=float(rng.uniform(0.05, 0.5)))
        lv = levels_of(cols)
        run_sweep(rng, cols, lv, nw=8, mb=int(rng.choice([2, 4, 8])))


@pytest.mark.parametrize("seed", range(6))
def test_factorization_waits(seed):
    rng = np.random.default_rng(100 + seed)
    for trial in range(20):
        n = int(rng.integers(20, 120))
        cols = random_pattern(rng, n, band=int(rng.integers(3, 25)), density=float(rng.uniform(0.05, 0.5)))
        lv = levels_of(cols)
        run_factor(rng, cols, lv, nw=int(rng.integers(1, 5)))


def test_model_catches_a_broken_rule():
    """The checks have teeth: with tasks allowed to run one phase early, some interleaving
    reads a row before it is written."""
    rng = np.random.default_rng(7)
    cols = random_pattern(rng, 60, band=8, density=0.3)
    lv = levels_of(cols)
    for s in range(50):  # the correct rule never fails here
        run_sweep(np.random.default_rng(s), cols, lv, 8, 4)
    with pytest.raises(AssertionError):
        for s in range(50):
            run_sweep(np.random.default_rng(s), cols, lv, 8, 4, early=1)
