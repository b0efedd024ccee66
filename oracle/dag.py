"""Access-mode dependency inference and task lists, written plainly in Python.

TEST INFRASTRUCTURE ONLY (see ``oracle/core.py``).

Section 2 of the paper states that the access modes of a task's buffer
parameters (read-only, write-only, read-write) together with the sequence of
task invocations determine the dependency graph.  The reading used here:

* a task that reads a datum depends on the last task that wrote it (RAW);
* a task that writes a datum depends on the last writer (WAW) and on every
  task that read it since that write (WAR), and then becomes its last writer.

Write-only (``W``) follows the same ordering rules as read-write; its only
difference is that the previous contents need not be read.

The tiled Cholesky tasks are listed in the right-looking order used by the
sequential program (Section 5.1 names Cholesky as the partitioning idiom):
for each k, POTRF(k); TRSM(i,k) for i>k; then for each i>k, SYRK(i,k)
followed by GEMM(i,j,k) for k<j<i.  The solve lists the forward sweep
(TRSM_L(K) then GEMM_RHS_N(I,K) for I>K, K ascending) and the backward sweep
(TRSM_LT(K) then GEMM_RHS_T(I,K) for I<K, K descending).
"""
import random

R, W, RW = 1, 2, 3

# kind names shared with oracle/core.py's integer codes
POTRF, TRSM, SYRK, GEMM, TRSM_L, GEMM_RHS_N, TRSM_LT, GEMM_RHS_T = range(8)


def cholesky_tasks(t):
    """Factor tasks in submission order: (kind, (i, j, k), [(datum, mode)])."""
    tasks = []
    for k in range(t):
        tasks.append((POTRF, (k, 0, 0), [(("A", k, k), RW)]))
        for i in range(k + 1, t):
            tasks.append((TRSM, (i, 0, k), [(("A", k, k), R), (("A", i, k), RW)]))
        for i in range(k + 1, t):
            tasks.append((SYRK, (i, 0, k), [(("A", i, k), R), (("A", i, i), RW)]))
            for j in range(k + 1, i):
                tasks.append((GEMM, (i, j, k), [(("A", i, k), R), (("A", j, k), R),
                                                (("A", i, j), RW)]))
    return tasks


def solve_tasks(t):
    """Forward then backward solve tasks on RHS blocks B_0..B_{t-1}."""
    tasks = []
    for k in range(t):
        tasks.append((TRSM_L, (k, 0, 0), [(("A", k, k), R), (("B", k), RW)]))
        for i in range(k + 1, t):
            tasks.append((GEMM_RHS_N, (i, 0, k), [(("A", i, k), R), (("B", k), R),
                                                   (("B", i), RW)]))
    for k in range(t - 1, -1, -1):
        tasks.append((TRSM_LT, (k, 0, 0), [(("A", k, k), R), (("B", k), RW)]))
        for i in range(k - 1, -1, -1):
            tasks.append((GEMM_RHS_T, (i, 0, k), [(("A", k, i), R), (("B", k), R),
                                                   (("B", i), RW)]))
    return tasks


def infer_dag(tasks):
    """Returns (preds, succs, war_edges): lists of sets of task indices, and
    the set of edges that exist only because of a write-after-read."""
    n = len(tasks)
    preds = [set() for _ in range(n)]
    last_writer = {}
    readers = {}
    war = set()
    for t, (_, _, acc) in enumerate(tasks):
        for datum, mode in acc:
            lw = last_writer.get(datum)
            if mode & W:
                if lw is not None:
                    preds[t].add(lw)
                for rd in readers.get(datum, ()):
                    if rd != t:
                        preds[t].add(rd)
                        if rd != lw:
                            war.add((rd, t))
            elif lw is not None:
                preds[t].add(lw)
        for datum, mode in acc:
            if mode & W:
                last_writer[datum] = t
                readers[datum] = []
            else:
                readers.setdefault(datum, []).append(t)
    succs = [set() for _ in range(n)]
    for t in range(n):
        for p in preds[t]:
            succs[p].add(t)
    # a WAR edge also implied by a RAW/WAW path is still reported; callers
    # only test for its presence or absence
    return preds, succs, war


def random_topological_order(preds, succs, rng):
    """Kahn's algorithm with a random choice among the ready tasks."""
    indeg = [len(p) for p in preds]
    ready = [t for t, d in enumerate(indeg) if d == 0]
    order = []
    while ready:
        t = ready.pop(rng.randrange(len(ready)))
        order.append(t)
        for s in succs[t]:
            indeg[s] -= 1
            if indeg[s] == 0:
                ready.append(s)
    if len(order) != len(preds):
        raise ValueError("dependency graph has a cycle")
    return order


def critical_path_length(preds):
    """Number of tasks on the longest dependency chain (tasks are listed in a
    topological order: submission order always is one)."""
    depth = []
    for t, p in enumerate(preds):
        depth.append(1 + max((depth[q] for q in p), default=0))
    return max(depth, default=0)


def is_valid_order(order, preds):
    pos = {t: i for i, t in enumerate(order)}
    return all(pos[p] < pos[t] for t in range(len(preds)) for p in preds[t])


def make_rng(seed):
    return random.Random(seed)
