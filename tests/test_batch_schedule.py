"""CPU emulation of the persistent batched launch's schedule (no GPU).

The kernel runs S steps of every grid in one launch: workgroup w (after the
XCD-aware renumbering of the hardware workgroup index) takes items w, w + G,
w + 2G, ... of a step's item table, then every workgroup meets at a
grid-wide barrier whose protocol is: the control block's count and
generation are cleared before the launch; at barrier s a workgroup adds
itself to the count; the last to arrive clears the count and publishes
generation s + 1; the others wait until the generation reaches s + 1.  The
emulation runs the workgroups as threads with random delays, through
several launches in a row (graph replays), and checks what the kernel
relies on: the renumbering is a permutation of the workgroups, every item
of every step runs exactly once, no item of step s + 1 starts before every
item of step s has finished, every workgroup passes the same number of
barriers, and the buffer parity each item uses equals that of plain
stepping.
"""
import random
import threading

import pytest


def xcd_remap(bid: int, nb: int) -> int:
    """The kernel's XCD-aware renumbering (workgroups are dealt round-robin
    over the 8 XCDs; each XCD gets a contiguous range of logical indices)."""
    q, r = divmod(nb, 8)
    x, l = bid % 8, bid // 8
    return (x * (q + 1) if x < r else r * (q + 1) + (x - r) * q) + l


@pytest.mark.parametrize("nb", list(range(1, 70)) + [255, 256, 512, 1000, 2048])
def test_renumbering_is_a_permutation(nb):
    assert sorted(xcd_remap(b, nb) for b in range(nb)) == list(range(nb))


class Ctl:
    """Control block: step base, buffer flips, barrier count and generation."""

    def __init__(self):
        self.lock = threading.Condition()
        self.step_base = 0
        self.flip = 0
        self.count = 0
        self.gen = 0


def _launch(ctl, G, P, S, item_grid, par0, log, clock):
    # k_batch_bar_reset before the launch
    ctl.count, ctl.gen = 0, 0
    base, flip = ctl.step_base, ctl.flip
    barriers = [0] * G

    def workgroup(bid):
        rnd = random.Random(bid * 7919 + base)
        w = xcd_remap(bid, G)
        for s in range(S):
            for r in range(w, P, G):
                g = item_grid[r]
                with ctl.lock:
                    start = next(clock)
                if rnd.random() < 0.3:
                    threading.Event().wait(rnd.random() * 1e-3)
                with ctl.lock:
                    log.append((base + s, r, (par0[g] + flip + s) & 1, start, next(clock)))
            # barrier s: arrive, last one publishes generation s + 1
            with ctl.lock:
                ctl.count += 1
                if ctl.count == G:
                    ctl.count = 0
                    ctl.gen = s + 1
                    ctl.lock.notify_all()
                else:
                    while ctl.gen < s + 1:
                        ctl.lock.wait(timeout=5.0)
                        assert ctl.gen >= s + 1 or ctl.count < G
            barriers[bid] += 1

    th = [threading.Thread(target=workgroup, args=(b,)) for b in range(G)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=60)
        assert not t.is_alive(), "emulated launch did not finish"
    assert barriers == [S] * G
    # one thread of workgroup 0 advances the control block after the last barrier
    ctl.step_base = base + S
    ctl.flip = flip + S


@pytest.mark.parametrize("G,P,S,launches", [(1, 5, 4, 2), (7, 30, 5, 3), (16, 16, 3, 2),
                                             (13, 100, 4, 2), (32, 9, 3, 1)])
def test_persistent_schedule(G, P, S, launches):
    import itertools
    rng = random.Random(G * 1000 + P)
    ngrids = 4
    item_grid = sorted(rng.randrange(ngrids) for _ in range(P))
    par0 = [0] * ngrids
    ctl = Ctl()
    log = []
    clock = itertools.count()
    for _ in range(launches):
        _launch(ctl, min(G, P), P, S, item_grid, par0, log, clock)
    total = S * launches
    seen = {}
    for step, r, parity, start, end in log:
        assert (step, r) not in seen, "item ran twice in a step"
        seen[(step, r)] = (start, end)
        assert parity == step & 1       # plain stepping swaps the sets once per step
    assert len(seen) == total * P       # every item of every step ran
    for step in range(total - 1):
        last_end = max(seen[(step, r)][1] for r in range(P))
        first_next = min(seen[(step + 1, r)][0] for r in range(P))
        assert last_end < first_next, f"step {step + 1} started before step {step} finished"
    assert ctl.step_base == total and ctl.flip == total
