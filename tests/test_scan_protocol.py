"""Model of the scan block's meeting protocol (CPU, random interleavings).

The scan's 16 waves walk their share of each round (at most 64 inserted
keys per wave and round: one entry per lane) at their own pace; a wave checks
the buffer count after each of its rounds and waits at a meeting when the
count is above T = cap - 1024 or when it has finished.  At a meeting every wave reads the
same decision (cut back, or all done).  A cut-back first keeps the keys whose
distance is at most the n-th smallest distance (ties may keep more than n),
and cuts exactly to n only when that would still leave more than T: so it
leaves between n and T keys, which the model draws at random.
The model interleaves the waves' steps at random and checks what the kernel
relies on: the count never exceeds cap, every meeting gathers all waves,
every round of every wave is walked once, and the loop ends.
"""
import random

import pytest

WAVES, PER_WAVE, ROUND = 16, 64, 1024


def _run(seed, rounds, cap, n):
    rng = random.Random(seed)
    T = cap - ROUND
    done = [rounds == 0] * WAVES
    counted = [False] * WAVES
    walked = [0] * WAVES
    state = ["next"] * WAVES
    pending = [0] * WAVES
    waiting = set()
    count = done_waves = meetings = peak = 0
    p_pass = 1.0
    for _ in range(5_000_000):
        runnable = [w for w in range(WAVES) if w not in waiting]
        if not runnable:  # every wave waits: the meeting takes place
            meetings += 1
            if done_waves == WAVES:
                return peak, meetings, walked
            if count > T:
                count = rng.randint(min(count, n), min(count, T))  # loose or exact cut
                p_pass = max(0.01, p_pass * 0.5)
            waiting.clear()
            state = ["next"] * WAVES
            continue
        w = rng.choice(runnable)
        if state[w] == "next":
            if done[w]:
                state[w] = "check"
            else:
                pending[w] = sum(rng.random() < p_pass for _ in range(PER_WAVE))
                state[w] = "insert"
        elif state[w] == "insert":  # inserts land in pieces, interleaved with other waves
            k = min(pending[w], rng.randint(0, 64))
            count += k
            pending[w] -= k
            peak = max(peak, count)
            if pending[w] == 0:
                walked[w] += 1
                done[w] = walked[w] >= rounds
                state[w] = "check"
        else:  # check: meet when done or when the count is above T
            if done[w] or count > T:
                if done[w] and not counted[w]:
                    counted[w] = True
                    done_waves += 1
                waiting.add(w)
            else:
                state[w] = "next"
    raise AssertionError("the loop did not end")


@pytest.mark.parametrize("n", [1, 10, 200, 1400, 2400])
def test_meeting_protocol_bounds_and_termination(n):
    rng = random.Random(n)
    for trial in range(150):
        rounds = rng.randint(0, 50)
        cap = n + ROUND + rng.choice([0, 64, 512, 2048])
        peak, meetings, walked = _run(1000 * n + trial, rounds, cap, n)
        assert peak <= cap, (n, trial, peak, cap)
        assert walked == [rounds] * WAVES
        assert meetings >= 1
