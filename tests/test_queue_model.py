"""Model of the persistent batch's device queue (CPU, no GPU).

The protocol of persistent_batch_kernel (paper_2111_14641_amd/csrc/
batch_kernels.hip), restated step by step: each workgroup reads the head,
looks at 64 slots from it at once (queued?, every item taken?), takes an item
of the first stage with items left by an atomic add, and moves the head by an
atomic max to the end of the exhausted prefix (past the stage taken when it is
that end and its last item was taken); the workgroup that finishes a stage's
last item reserves a slot (atomic add on the tail) and publishes the successor
stage later.  A random scheduler interleaves the workgroups' steps, with the
gap between a slot's reservation and its publication, and between a
workgroup's look at the slots and its atomic add, as wide as it likes.  Every
item of every stage must be taken exactly once, every problem must finish,
and the head must never pass a stage that is not queued or has items left."""
import random

import pytest


class Queue:
    def __init__(self, chains):
        self.chains = chains                     # per problem: item counts of its stages
        self.total = sum(len(c) for c in chains)
        self.stage = [None] * self.total         # (problem, index in chain)
        self.valid = [0] * self.total
        self.claimed = [0] * self.total
        self.finished = [0] * self.total
        self.taken = [0] * self.total            # successful claims (checked)
        self.head = 0
        self.tail = 0
        self.done = 0
        for q in range(len(chains)):
            self.publish(self.reserve(), (q, 0))

    def n(self, slot):
        q, i = self.stage[slot]
        return self.chains[q][i]

    def reserve(self):
        t = self.tail
        self.tail += 1
        assert t < self.total
        return t

    def publish(self, t, st):
        self.stage[t] = st
        self.valid[t] = 1

    def check_head(self):
        for s in range(min(self.head, self.total)):
            assert self.valid[s] and self.claimed[s] >= self.n(s), f"head passed slot {s}"


def workgroup(Q, rng):
    """A generator: one yield per shared-memory step of one workgroup."""
    while True:
        # --- claim --------------------------------------------------------
        while True:
            h0 = Q.head
            yield
            if h0 >= Q.total:
                return
            window = []
            for lane in range(64):
                s = h0 + lane
                if s >= Q.total:
                    window.append((False, False, 0))
                    continue
                queued = bool(Q.valid[s])
                n = Q.n(s) if queued else 0
                left = queued and Q.claimed[s] < n
                window.append((queued, left, n))
            yield
            g = next((i for i, (qd, lf, _) in enumerate(window) if not (qd and not lf)), 64)
            f = next((i for i, (_, lf, _) in enumerate(window) if lf), None)
            if f is None:
                if g > 0:
                    Q.head = max(Q.head, h0 + g)
                    Q.check_head()
                yield
                continue
            hs, nf = h0 + f, window[f][2]
            c = Q.claimed[hs]
            Q.claimed[hs] += 1
            yield
            if c >= nf:
                continue
            Q.taken[hs] += 1
            nxt = hs + 1 if (f == g and c + 1 == nf) else h0 + g
            if nxt > h0:
                Q.head = max(Q.head, nxt)
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
                t = Q.reserve()
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
    assert Q.tail == Q.total
    for s in range(Q.total):
        assert Q.taken[s] == Q.n(s), (s, Q.taken[s], Q.n(s))
    assert Q.head == Q.total


def test_model_catches_a_head_moved_past_an_unqueued_stage():
    """The model must flag the mistake of moving the head to the stage taken
    (past every slot before it) without checking that those slots are
    exhausted: with reservations published late, some seed makes a workgroup
    take a later stage while an earlier slot is still unpublished."""
    def bad_workgroup(Q, rng):
        while True:
            while True:
                h0 = Q.head
                yield
                if h0 >= Q.total:
                    return
                f = None
                for lane in range(64):
                    s = h0 + lane
                    if s < Q.total and Q.valid[s] and Q.claimed[s] < Q.n(s):
                        f = lane
                        break
                yield
                if f is None:
                    yield
                    continue
                hs, nf = h0 + f, Q.n(h0 + f)
                c = Q.claimed[hs]
                Q.claimed[hs] += 1
                if c >= nf:
                    continue
                Q.taken[hs] += 1
                Q.head = max(Q.head, hs + 1 if c + 1 == nf else hs)   # the mistake
                Q.check_head()
                yield
                break
            yield
            Q.finished[hs] += 1
            if Q.finished[hs] == nf:
                q, i = Q.stage[hs]
                if i + 1 < len(Q.chains[q]):
                    t = Q.reserve()
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
