"""CPU model of the persistent QR's column-slot ring (no GPU).

In the persistent factorization without pivoting, workgroup w owns columns
w*CPG .. (w+1)*CPG-1.  At step i every workgroup needs column i: it waits for
a record (all G records of step i at an exchange step, only the owner's
record otherwise), reads the column from the owner's slot i mod R, updates,
and publishes its record for step i+1; the owner of column i+1 also writes
that column into its slot (i+1) mod R.  A slot is rewritten R steps after it
was filled, so the rule "exchange at every step that is a multiple of R/2"
must guarantee that every workgroup has read a slot before its owner fills
it again.  The kernel itself cannot show that for every interleaving (a
rewritten slot carries a newer step tag, so a late reader would only spin
until its bounded wait gives up), so this test checks the rule on random
schedules of a model of the protocol, and checks that a rule with too few
exchanges for the ring is caught.
"""
import random

import pytest


def run_schedule(G, CPG, K, R, E, seed):
    """One random interleaving of G workgroups over K steps with R slots per
    workgroup and a full exchange at every step that is a multiple of E.
    Returns None on success, or a description of the first stale read."""
    rng = random.Random(seed)
    records = [set() for _ in range(K + 1)]  # records[i]: workgroups that published step i
    slots = {}  # (owner, slot) -> step of the column it holds
    step = [0] * G  # next step of each workgroup
    phase = [0] * G  # 0: publish(step), 1: gather + read + update

    def owner(i):
        return i // CPG

    while True:
        ready = []
        for w in range(G):
            i = step[w]
            if i >= K:
                continue
            if phase[w] == 0:
                ready.append(w)
                continue
            full = E == 1 or i % E == 0
            need = range(G) if full else (owner(i),)
            if all(x in records[i] for x in need):
                ready.append(w)
        if not ready:
            if all(s >= K for s in step):
                return None
            return f"deadlock at steps {step}"
        w = rng.choice(ready)
        i = step[w]
        if phase[w] == 0:
            records[i].add(w)
            if owner(i) == w:
                slots[(w, i % R)] = i
            phase[w] = 1
        else:
            held = slots.get((owner(i), i % R))
            if held != i:
                return f"workgroup {w} read slot {i % R} of workgroup {owner(i)} at step {i}: holds step {held}"
            step[w] = i + 1
            phase[w] = 0


@pytest.mark.parametrize("R", [2, 4, 8])
@pytest.mark.parametrize("G,CPG", [(2, 2), (3, 1), (5, 3), (8, 8)])
def test_ring_rule_never_reads_a_rewritten_slot(R, G, CPG):
    """The kernel's rule: R slots, full exchange every R/2 steps (every step
    for R = 2).  Random schedules, biased by the random choice among the
    workgroups that may move, never read a rewritten slot and never stall."""
    E = max(1, R // 2)
    K = G * CPG
    for seed in range(150):
        assert run_schedule(G, CPG, K, R, E, seed) is None, (R, G, CPG, seed)


def test_too_few_exchanges_for_the_ring_are_caught():
    """A rule with an exchange only every R steps (E = R) lets an owner of
    consecutive columns run a full ring ahead: some schedule reads a slot
    its owner has filled again.  The model must find one."""
    found = [run_schedule(4, 8, 32, 4, 4, seed) for seed in range(300)]
    assert any(f is not None and "holds step" in f for f in found)


def test_no_exchange_between_owner_steps_is_caught():
    """Two slots without an exchange at every step (the rule the pivoting
    launches keep) fail as well."""
    found = [run_schedule(3, 4, 12, 2, 2, seed) for seed in range(300)]
    assert any(f is not None and "holds step" in f for f in found)
