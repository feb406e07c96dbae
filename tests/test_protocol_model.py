"""Exhaustive interleaving check of the dual-mailbox protocol model (the dispatch
oracle) and of its Table 1 codes against the values the paper prints."""
import os

import pytest

from oracle import protocol_model as pm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_mailbox_codes.txt")


def _golden_codes():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        d, name, v = line.split()
        out[(d, name)] = int(v)
    return out


def test_model_codes_are_table1():
    g = _golden_codes()
    assert g[("from_GPU", "THREAD_INIT")] == pm.FROM_INIT
    assert g[("from_GPU", "THREAD_FINISHED")] == pm.FROM_FINISHED
    assert g[("from_GPU", "THREAD_WORKING")] == pm.FROM_WORKING
    assert g[("from_GPU", "THREAD_NOP")] == pm.FROM_NOP
    assert g[("to_GPU", "THREAD_NOP")] == pm.TO_NOP
    assert g[("to_GPU", "THREAD_EXIT")] == pm.TO_EXIT
    assert g[("to_GPU", "THREAD_WORK")] == pm.TO_WORK


SYSTEMS = [
    pm.Config(((0,),), (0, 0, 0), 1),
    pm.Config(((0,),), (0, 0, 0), 2),
    pm.Config(((0,), (1,)), (0, 1, 0, 1), 1),
    pm.Config(((0,), (1,)), (0, 0, 1, 0), 2),
    pm.Config(((0, 1),), (0, 0, 0), 1),
    pm.Config(((0, 1),), (0, 0, 0), 2),
    pm.Config(((0, 1), (2,)), (0, 1, 0), 1),
]


@pytest.mark.parametrize("cfg", SYSTEMS, ids=lambda c: f"{c.clusters}-{c.items}-d{c.depth}")
def test_protocol_holds_on_every_interleaving(cfg):
    n = pm.check(cfg)
    assert n > 10


@pytest.mark.parametrize("bug,expect", [
    ("cmd_before_payload", "I1"),       # doorbell published before the descriptor
    ("status_before_output", "I4"),     # completion published before the output
    ("no_ring_check", "deadlock"),      # host overwrites an unconsumed slot
    ("no_seq", "I1"),                   # bare code word without sequence number
])
def test_checker_catches_planted_protocol_bugs(bug, expect):
    caught = 0
    for cfg in SYSTEMS[2:]:
        bad = pm.Config(cfg.clusters, cfg.items, cfg.depth, bug)
        try:
            pm.check(bad)
        except pm.Violation as e:
            assert str(e).startswith(expect), str(e)
            caught += 1
    assert caught >= 3


LOOKAHEAD_SYSTEMS = [
    pm.Config(((0,),), (0, 0, 0), 2, lookahead=True),
    pm.Config(((0,),), (0, 0, 0, 0), 3, lookahead=True),
    pm.Config(((0,), (1,)), (0, 0, 1, 0), 2, lookahead=True),
    pm.Config(((0, 1),), (0, 0, 0), 2, lookahead=True),
]


@pytest.mark.parametrize("cfg", LOOKAHEAD_SYSTEMS, ids=lambda c: f"{c.clusters}-{c.items}-d{c.depth}-ahead")
def test_protocol_holds_with_the_lookahead_read(cfg):
    """A worker may snapshot its next slot at any point while it runs an item and take
    the command from the snapshot when its sequence number is the expected one: every
    property still holds on every interleaving (the ring check keeps the slot from being
    reused before the snapshot's command has run)."""
    n = pm.check(cfg)
    assert n > pm.check(pm.Config(cfg.clusters, cfg.items, cfg.depth))  # the snapshots add states


def test_checker_catches_a_lookahead_without_sequence_check():
    caught = 0
    for cfg in LOOKAHEAD_SYSTEMS:
        bad = pm.Config(cfg.clusters, cfg.items, cfg.depth, "ahead_no_seq", lookahead=True)
        try:
            pm.check(bad)
        except pm.Violation as e:
            assert str(e).startswith("I"), str(e)
            caught += 1
    assert caught == len(LOOKAHEAD_SYSTEMS)

