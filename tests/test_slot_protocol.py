"""Model check of the cross-wave summation protocol of the Legendre adjoint kernel.

The kernel's waves of one workgroup sum their per-chunk results without workgroup barriers:
for round r a wave waits until slot r % S has been handed on r // S times, adds its values
into the slot (LDS atomics), and counts itself in; the live wave whose count completes the
round adds the slot into the output, clears it, resets the count and hands the slot on.
This host model runs the same protocol, one LDS operation per step, under random and
adversarial interleavings of the waves, and checks that every run ends (no wave waits
forever) and that every round's sum reaches the output exactly once.  The kernel's bound on
the wait is not modelled: the model shows it is never reached.
"""
import random

import pytest


def run_protocol(nlive, nrounds, nslots, pick, max_steps=200000):
    """Simulate nlive waves; pick(ready) chooses which runnable wave takes the next step."""
    slot = [dict() for _ in range(nslots)]   # round -> summed value, per slot
    cnt = [0] * nslots
    gen = [0] * nslots
    out = {}
    # per-wave program counter: (round, phase)
    state = [[0, "wait"] for _ in range(nlive)]
    steps = 0
    while any(st[0] < nrounds for st in state):
        ready = []
        for w, (r, ph) in enumerate(state):
            if r >= nrounds:
                continue
            s = r % nslots
            if ph == "wait" and gen[s] != r // nslots:
                continue  # spinning: no progress possible this step
            ready.append(w)
        assert ready, "deadlock: every unfinished wave waits for a slot"
        w = pick(ready)
        r, ph = state[w]
        s = r % nslots
        if ph == "wait":
            state[w][1] = "add"
        elif ph == "add":
            # values of different rounds in one slot would be a protocol error
            assert all(k == r for k in slot[s]), "slot holds another round's values"
            slot[s][r] = slot[s].get(r, 0) + (w + 1) * 1000 + r
            state[w][1] = "count"
        elif ph == "count":
            arrived = cnt[s]
            cnt[s] += 1
            if arrived == nlive - 1:
                state[w][1] = "flush"
            else:
                state[w] = [r + 1, "wait"]
        elif ph == "flush":
            assert r not in out, "round flushed twice"
            out[r] = slot[s].pop(r)
            cnt[s] = 0
            gen[s] += 1
            state[w] = [r + 1, "wait"]
        steps += 1
        assert steps < max_steps
    return out


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
