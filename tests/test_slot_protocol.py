"""Model check of the cross-wave summation protocol of the Legendre adjoint kernel.

The kernel's waves of one workgroup sum their per-chunk results without workgroup barriers:
for round r a wave waits until slot r % S has been handed on r // S times, adds its values
into the slot (LDS atomics), and counts itself in; the live wave whose count completes the
round adds the slot into the output, clears it, resets the count and hands the slot on.
This host model runs the same protocol, one LDS operation per step, under random and
adversarial interleavings of the waves, and checks that every run ends (no wave waits
forever) and that every round's sum reaches the output exactly once.  With the kernel's bound
on the wait modelled (a waiting wave that has spun `spin_limit` times goes on and sets the
error word that the host turns into NUSHT_EDEVICE), it also checks that a run whose word
stays clear summed every round exactly once, and that a broken hand-on ends with the word set
instead of hanging.
"""
import random

import pytest


def run_protocol(nlive, nrounds, nslots, pick, max_steps=200000, spin_limit=None,
                 hand_on=True, with_flag=False):
    """Simulate nlive waves; pick(ready) chooses which runnable wave takes the next step.

    spin_limit=None: a waiting wave makes no progress until its slot is handed on (the model
    asserts that some wave can always move).  Otherwise a waiting wave spins one step at a
    time and, after spin_limit spins, goes on and sets the error word.  hand_on=False plants
    a broken flush that never hands the slot on.  Returns the flushed rounds (and the error
    word if with_flag)."""
    slot = [dict() for _ in range(nslots)]   # round -> summed value, per slot
    cnt = [0] * nslots
    gen = [0] * nslots
    out = {}
    err = 0
    # per-wave program counter: (round, phase, spins)
    state = [[0, "wait", 0] for _ in range(nlive)]
    steps = 0
    while any(st[0] < nrounds for st in state):
        ready = []
        for w, (r, ph, _) in enumerate(state):
            if r >= nrounds:
                continue
            s = r % nslots
            if ph == "wait" and gen[s] != r // nslots and spin_limit is None:
                continue  # spinning: no progress possible this step
            ready.append(w)
        assert ready, "deadlock: every unfinished wave waits for a slot"
        w = pick(ready)
        r, ph, spins = state[w]
        s = r % nslots
        if ph == "wait":
            if gen[s] == r // nslots:
                state[w][1] = "add"
            elif spins + 1 >= spin_limit:
                err |= 1                      # the wait gave up: flagged, then goes on
                state[w][1] = "add"
            else:
                state[w][2] = spins + 1
        elif ph == "add":
            if any(k != r for k in slot[s]):
                # another round's values still in the slot: only after a give-up
                assert err, "slot holds another round's values"
            slot[s][r] = slot[s].get(r, 0) + (w + 1) * 1000 + r
            state[w][1] = "count"
        elif ph == "count":
            arrived = cnt[s]
            cnt[s] += 1
            if arrived == nlive - 1:
                state[w][1] = "flush"
            else:
                state[w] = [r + 1, "wait", 0]
        elif ph == "flush":
            # after a give-up the counts mix rounds and sums are wrong (flagged); before it
            # every round is flushed once
            assert err or r not in out, "round flushed twice"
            out[r] = slot[s].pop(r, None)
            for k in list(slot[s]):
                out.setdefault(k, None)       # mixed rounds: the sums are wrong
                slot[s].pop(k)
            cnt[s] = 0
            if hand_on:
                gen[s] += 1
            state[w] = [r + 1, "wait", 0]
        steps += 1
        assert steps < max_steps
    return (out, err) if with_flag else out


def expected(nlive, nrounds):
    return {r: sum((w + 1) * 1000 + r for w in range(nlive)) for r in range(nrounds)}


@pytest.mark.parametrize("nslots", [1, 2, 4])
@pytest.mark.parametrize("nlive", [1, 2, 3, 4])
def test_random_interleavings_end_with_every_round_summed_once(nlive, nslots):
    for seed in range(200):
        rng = random.Random(seed * 31 + nlive * 7 + nslots)
        out = run_protocol(nlive, 9, nslots, lambda ready: rng.choice(ready))
        assert out == expected(nlive, 9)


@pytest.mark.parametrize("nslots", [1, 2, 4])
def test_one_wave_racing_ahead_waits_and_never_deadlocks(nslots):
    # wave 0 always moves when it can; the others only when it cannot
    out = run_protocol(4, 12, nslots, lambda ready: 0 if 0 in ready else ready[-1])
    assert out == expected(4, 12)
    # the slowest wave is starved as long as any other can move
    out = run_protocol(4, 12, nslots, lambda ready: max(ready) if len(ready) > 1 else ready[0])
    assert out == expected(4, 12)


@pytest.mark.parametrize("nslots", [1, 2])
def test_bounded_wait_flags_every_give_up_and_clean_runs_are_exact(nslots):
    """A tiny bound makes waves give up under random interleavings: every run ends, and every
    run whose error word stays clear has summed each round exactly once."""
    clean = flagged = 0
    for seed in range(300):
        rng = random.Random(seed)
        out, err = run_protocol(4, 9, nslots, lambda ready: rng.choice(ready), spin_limit=10,
                                with_flag=True)
        if err:
            flagged += 1
        else:
            clean += 1
            assert out == expected(4, 9)
    assert flagged > 0 and clean > 0


def test_broken_hand_on_ends_with_the_error_word_set():
    """A flush that never hands the slot on would hang the waves of later rounds; with the
    bound they go on and the error word is set (NUSHT_EDEVICE on the host)."""
    with pytest.raises(AssertionError, match="deadlock"):
        run_protocol(4, 6, 2, lambda ready: ready[0], hand_on=False)
    out, err = run_protocol(4, 6, 2, lambda ready: ready[0], spin_limit=50, hand_on=False,
                            with_flag=True)
    assert err == 1


def test_generous_bound_is_never_reached():
    for seed in range(100):
        rng = random.Random(1000 + seed)
        out, err = run_protocol(4, 9, 2, lambda ready: rng.choice(ready), spin_limit=10 ** 6,
                                with_flag=True)
        assert err == 0 and out == expected(4, 9)
