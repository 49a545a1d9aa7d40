"""Model of the persistent batch's device queue (CPU, no GPU).

The protocol of persistent_batch_kernel (paper_2111_14641_amd/csrc/
batch_kernels.hip), restated step by step.  The queue has priority levels, each
a FIFO over its own range of slots.  Each workgroup reads every level's head,
looks at 16 slots from each at once (queued?, every item taken?), takes an item
of the first stage with items left (highest level first) by an atomic add, and
moves that level's head by an atomic max to the end of its exhausted prefix
(past the stage taken when it is that end and its last item was taken); the
workgroup that finishes a stage's last item reserves a slot in the successor's
level (atomic add on that level's tail) and publishes the successor later.
A random scheduler interleaves the workgroups' steps, with the gap between a
slot's reservation and its publication, and between a workgroup's look at the
slots and its atomic add, as wide as it likes.  Every
item of every stage must be taken exactly once, every problem must finish,
and the head must never pass a stage that is not queued or has items left."""
import random

import pytest


LEVELS = 4
WINDOW = 16


def level_of(chain, i):
    """Priority of stage i of a chain: grows with the stages left."""
    return min(LEVELS - 1, (len(chain) - i - 1) // 4)


class Queue:
    def __init__(self, chains):
        self.chains = chains                     # per problem: item counts of its stages
        self.total = sum(len(c) for c in chains)
        need = [0] * LEVELS
        for c in chains:
            for i in range(len(c)):
                need[level_of(c, i)] += 1
        self.base, self.end = [], []
        b = 0
        for lv in range(LEVELS):
            self.base.append(b)
            b += need[lv]
            self.end.append(b)
        self.head = list(self.base)
        self.tail = list(self.base)
        self.stage = [None] * self.total         # (problem, index in chain)
        self.valid = [0] * self.total
        self.claimed = [0] * self.total
        self.finished = [0] * self.total
        self.taken = [0] * self.total            # successful claims (checked)
        self.done = 0
        for q in range(len(chains)):
            self.publish(self.reserve(level_of(chains[q], 0)), (q, 0))

    def n(self, slot):
        q, i = self.stage[slot]
        return self.chains[q][i]

    def reserve(self, lv):
        t = self.tail[lv]
        self.tail[lv] += 1
        assert t < self.end[lv]
        return t

    def publish(self, t, st):
        self.stage[t] = st
        self.valid[t] = 1

    def check_head(self):
        for lv in range(LEVELS):
            for s in range(self.base[lv], min(self.head[lv], self.end[lv])):
                assert self.valid[s] and self.claimed[s] >= self.n(s), f"head passed slot {s}"


def workgroup(Q, rng):
    """A generator: one yield per shared-memory step of one workgroup."""
    while True:
        # --- claim --------------------------------------------------------
        while True:
            heads = list(Q.head)
            yield
            if all(heads[lv] >= Q.end[lv] for lv in range(LEVELS)):
                return
            window = []          # (level, slot, queued, left, n), highest level first
            for lv in reversed(range(LEVELS)):
                for i in range(WINDOW):
                    s = heads[lv] + i
                    if s >= Q.end[lv]:
                        window.append((lv, s, False, False, 0))
                        continue
                    queued = bool(Q.valid[s])
                    n = Q.n(s) if queued else 0
                    window.append((lv, s, queued, queued and Q.claimed[s] < n, n))
            yield
            g = {}
            for lv in range(LEVELS):
                grp = [w for w in window if w[0] == lv]
                g[lv] = next((i for i, w in enumerate(grp) if not (w[2] and not w[3])), WINDOW)
            pick = next((w for w in window if w[3]), None)
            if pick is None:
                for lv in range(LEVELS):
                    if g[lv] > 0:
                        Q.head[lv] = max(Q.head[lv], heads[lv] + g[lv])
                Q.check_head()
                yield
                continue
            lv, hs, _, _, nf = pick
            c = Q.claimed[hs]
            Q.claimed[hs] += 1
            yield
            if c >= nf:
                continue
            Q.taken[hs] += 1
            nxt = hs + 1 if (hs - heads[lv] == g[lv] and c + 1 == nf) else heads[lv] + g[lv]
            if nxt > heads[lv]:
                Q.head[lv] = max(Q.head[lv], nxt)
                Q.check_head()
            yield
            break
        # --- the item -------------------------------------------------------
        for _ in range(rng.randrange(1, 6)):
            yield
        # --- finish ---------------------------------------------------------
        Q.finished[hs] += 1
        last = Q.finished[hs] == nf
        yield
        if last:
            q, i = Q.stage[hs]
            if i + 1 < len(Q.chains[q]):
                t = Q.reserve(level_of(Q.chains[q], i + 1))
                for _ in range(rng.randrange(0, 8)):   # reserved, not yet published
                    yield
                Q.publish(t, (q, i + 1))
            else:
                Q.done += 1
            yield


@pytest.mark.parametrize("seed", range(40))
def test_queue_takes_every_item_once(seed):
    rng = random.Random(seed)
    nprob = rng.randrange(1, 40)
    chains = []
    for _ in range(nprob):
        nb = rng.randrange(1, 6)
        chain = [rng.randrange(1, 5), rng.randrange(1, 9), rng.randrange(1, 3)]
        for b in range(nb):
            chain += [1, rng.randrange(1, 7)]
            if b + 1 < nb:
                chain += [rng.randrange(1, 5), 1]
        chains.append(chain)
    Q = Queue(chains)
    nwg = rng.choice([1, 3, 16, 70])
    wgs = [workgroup(Q, random.Random(seed * 1000 + w)) for w in range(nwg)]
    alive = list(wgs)
    steps = 0
    while alive:
        w = rng.choice(alive)
        try:
            next(w)
        except StopIteration:
            alive.remove(w)
        steps += 1
        assert steps < 5_000_000, "no progress"
    assert Q.done == nprob
    assert Q.tail == Q.end
    for s in range(Q.total):
        assert Q.taken[s] == Q.n(s), (s, Q.taken[s], Q.n(s))
    assert Q.head == Q.end


def test_model_catches_a_head_moved_past_an_unqueued_stage():
    """The model must flag the mistake of moving a level's head to the stage
    taken (past every slot before it) without checking that those slots are
    exhausted: with reservations published late, some seed makes a workgroup
    take a later stage while an earlier slot is still unpublished."""
    def bad_workgroup(Q, rng):
        while True:
            while True:
                heads = list(Q.head)
                yield
                if all(heads[lv] >= Q.end[lv] for lv in range(LEVELS)):
                    return
                pick = None
                for lv in reversed(range(LEVELS)):
                    for i in range(WINDOW):
                        s = heads[lv] + i
                        if s < Q.end[lv] and Q.valid[s] and Q.claimed[s] < Q.n(s):
                            pick = (lv, s)
                            break
                    if pick:
                        break
                yield
                if pick is None:
                    yield
                    continue
                lv, hs = pick
                nf = Q.n(hs)
                c = Q.claimed[hs]
                Q.claimed[hs] += 1
                if c >= nf:
                    continue
                Q.taken[hs] += 1
                Q.head[lv] = max(Q.head[lv], hs + 1 if c + 1 == nf else hs)   # the mistake
                Q.check_head()
                yield
                break
            yield
            Q.finished[hs] += 1
            if Q.finished[hs] == nf:
                q, i = Q.stage[hs]
                if i + 1 < len(Q.chains[q]):
                    t = Q.reserve(level_of(Q.chains[q], i + 1))
                    for _ in range(rng.randrange(0, 8)):
                        yield
                    Q.publish(t, (q, i + 1))
                else:
                    Q.done += 1
            yield

    caught = 0
    for seed in range(30):
        rng = random.Random(seed)
        chains = [[1, 2, 1, 1, 2, 1, 1, 3] for _ in range(12)]
        Q = Queue(chains)
        wgs = [bad_workgroup(Q, random.Random(seed * 7 + w)) for w in range(16)]
        alive = list(wgs)
        try:
            steps = 0
            while alive and steps < 200_000:
                w = rng.choice(alive)
                try:
                    next(w)
                except StopIteration:
                    alive.remove(w)
                steps += 1
        except AssertionError:
            caught += 1
    assert caught > 0
