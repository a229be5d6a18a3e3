"""Index facts of the circle ordering that the inner eigensolver relies on
(64 indices, 32 pairs per step, 63 steps per sweep).  The SVD of Alg. 3
(Sec. "Singular Value Decomposition approach") is computed here by one-sided
block Jacobi, a method the paper leaves open; the pair ordering of its inner
64 x 64 eigensolver is the circle method.  Pair m of step s holds the indices
in slots m and 63 - m; slot 0 keeps index 0 and the others move one slot down
the ring 1..63 per step.
"""
import itertools

JP = 64


def slot_index(s, a):
    return 0 if a == 0 else ((a - 1 + s) % (JP - 1)) + 1


def pairs(s):
    return [tuple(sorted((slot_index(s, m), slot_index(s, JP - 1 - m)))) for m in range(JP // 2)]


def test_sweep_meets_every_pair_once():
    seen = [p for s in range(JP - 1) for p in pairs(s)]
    assert len(seen) == len(set(seen)) == JP * (JP - 1) // 2
    for s in range(JP - 1):  # each step is a perfect matching
        assert sorted(i for p in pairs(s) for i in p) == list(range(JP))


def test_next_step_pairs_lie_in_fixed_blocks():
    # pair m of step s + 1 takes its indices from pairs m - 1 and m + 1 of
    # step s ((0, 1) for m = 0, (30, 31) for m = 31): the 32 blocks whose
    # threads compute the next step's rotations
    for s in range(JP - 1):
        owner = {}
        for m, (i, j) in enumerate(pairs(s)):
            owner[i] = owner[j] = m
        for m, (i, j) in enumerate(pairs((s + 1) % (JP - 1))):
            blk = tuple(sorted((owner[i], owner[j])))
            want = (0, 1) if m == 0 else ((30, 31) if m == 31 else (m - 1, m + 1))
            assert blk == want, (s, m, blk)


def test_other_blocks_enumeration():
    # threads 32..495 take the remaining 464 blocks column by column
    fixed = {(0, 1), (30, 31)} | {(m - 1, m + 1) for m in range(1, 31)}
    got = []
    for t in range(32, 496):
        b, q = t - 32, 2
        while b >= (q - 1 if q < 31 else 29):
            b -= q - 1 if q < 31 else 29
            q += 1
        got.append((b + 1 if (q < 31 and b >= q - 2) else b, q))
    every = {(p, q) for q in range(1, 32) for p in range(q)}
    assert len(got) == len(set(got)) == 464
    assert set(got) | fixed == every and not set(got) & fixed


def test_lane_shifts_follow_the_slots():
    # R in registers: lane m holds slots m (top) and 63 - m (bottom); after a
    # step the new top of m is the old top of m + 1 (bottom of 31 for m = 31,
    # itself for m = 0) and the new bottom the old bottom of m - 1 (top of 1
    # for m = 0); the entries then sit in the next step's slots
    for s in range(JP - 1):
        top = [slot_index(s, m) for m in range(32)]
        bot = [slot_index(s, JP - 1 - m) for m in range(32)]
        ntop = [bot[31] if m == 31 else (top[0] if m == 0 else top[m + 1]) for m in range(32)]
        nbot = [top[1] if m == 0 else bot[m - 1] for m in range(32)]
        assert ntop == [slot_index(s + 1, m) for m in range(32)]
        assert nbot == [slot_index(s + 1, JP - 1 - m) for m in range(32)]
    # whole sweeps bring every index back to its own slot
    assert all(slot_index(JP - 1, a) == a for a in range(JP))


def test_slot_index_advances_by_one():
    for s, a in itertools.product(range(JP - 1), range(JP)):
        x = slot_index(s, a)
        nxt = 0 if x == 0 else (1 if x == JP - 1 else x + 1)
        assert slot_index(s + 1, a) == nxt
