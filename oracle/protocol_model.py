"""Exhaustive state-machine model of the dual-mailbox dispatch protocol.

TEST INFRASTRUCTURE ONLY.  It is the oracle for the *dispatch* semantics (as opposed to
the work-item arithmetic): a host and k persistent workers exchange commands and
statuses through per-worker mailboxes (Sec. 2.4, Fig. 2), with the command and status
codes of Table 1.  Table 1 gives values but no transitions, so the model fixes this
reading: every mailbox word carries a sequence number next to its code,
``word = (seq << 8) | code``; the host posts WORK (16 + op), NOP (4) or EXIT (8) commands
into a ring of ``depth`` slots (depth 1 is the paper's single slot); the worker answers
each command in the matching status slot with FINISHED (1) and, at boot, announces INIT (0).

Every interleaving of the atomic steps below is explored (depth-first search over the
reachable state graph) and these properties are checked:

  I1 exactly once   each posted (mailbox, seq) is executed exactly once;
  I2 FIFO           each worker executes seq 1, 2, 3, ... in order;
  I3 cluster only   an item posted to cluster c is executed only by members of c;
  I4 visibility     when the host observes an item complete, every member's output
                    for that item has been written;
  liveness          every reachable state that is not final has an enabled step, and
                    the final state (everything consumed, every worker exited) is
                    reachable from every reachable state.

With ``lookahead`` (depth > 1) a worker may also, at any point while it runs an item,
snapshot its next command slot once, and at its next poll take the command from that
snapshot when the snapshot holds the expected sequence number (the device's look-ahead
read, whose timing is left free here).

The ``bug`` argument plants a mistake in the model (never in the product) so that the
tests can show the checker catches each class of error.
"""
from dataclasses import dataclass
from typing import Tuple

# Table 1 codes (Sec. 2.4).
FROM_INIT, FROM_FINISHED, FROM_WORKING, FROM_NOP = 0, 1, 2, 4
TO_NOP, TO_EXIT, TO_WORK = 4, 8, 16

BUGS = ("none", "cmd_before_payload", "status_before_output", "no_ring_check", "no_seq", "ahead_no_seq")


@dataclass(frozen=True)
class Config:
    clusters: Tuple[Tuple[int, ...], ...]   # member worker ids per cluster
    items: Tuple[int, ...]                  # cluster id of each item, in host submission order
    depth: int = 1
    bug: str = "none"
    # look-ahead (depth > 1): while it runs an item a worker may snapshot its next slot
    # once, and take the command from that snapshot instead of reading the slot again
    # when the snapshot holds the expected sequence number
    lookahead: bool = False

    @property
    def n_workers(self):
        return 1 + max(w for c in self.clusters for w in c)


class Violation(AssertionError):
    pass


def _initial(cfg):
    W, D = cfg.n_workers, cfg.depth
    # cmd[w][s] = (seq, code, payload_item) where payload_item is the item index the
    # slot's payload describes (-1 = none); payload and word are written separately.
    cmd = tuple(tuple((0, TO_NOP, -1) for _ in range(D)) for _ in range(W))
    status = tuple(tuple((0, FROM_INIT) for _ in range(D)) for _ in range(W))
    # worker: (done_seq, phase, cur_item, exited, ahead) phase: 0 poll, 1 exec, 2 publish,
    # 3 exited; ahead = snapshot (seq, code, payload_item) of the next slot, or None
    workers = tuple((0, 0, -1, 0, None) for _ in range(W))
    outputs = frozenset()            # (item, worker) pairs whose output is written
    executed = ()                    # tuple of (worker, seq, item) in execution order
    # host: next item index to post, partially posted member index (-1 none),
    # per-cluster posted ticket and consumed ticket, exit posting progress
    n_c = len(cfg.clusters)
    host = (0, -1, tuple(0 for _ in range(n_c)), tuple(0 for _ in range(n_c)), -1, 0)
    return (cmd, status, workers, outputs, executed, host)


def _set(tup, i, v):
    return tup[:i] + (v,) + tup[i + 1:]


def _cluster_of(cfg, w):
    for c, members in enumerate(cfg.clusters):
        if w in members:
            return c
    raise ValueError


def _ticket_of_item(cfg, item):
    c = cfg.items[item]
    return sum(1 for i in range(item + 1) if cfg.items[i] == c)


def _item_of(cfg, c, ticket):
    k = 0
    for i, ci in enumerate(cfg.items):
        if ci == c:
            k += 1
            if k == ticket:
                return i
    return -1


def _steps(cfg, st):
    """Yield (label, next_state) for every enabled atomic step."""
    cmd, status, workers, outputs, executed, host = st
    D = cfg.depth
    nxt_item, stage, posted, consumed, exit_w, exit_stage = host

    # --- host: post the next item, member by member; each member takes two steps:
    #     write the payload, then publish the command word (release).
    if nxt_item < len(cfg.items) and exit_w < 0:
        c = cfg.items[nxt_item]
        members = cfg.clusters[c]
        t = posted[c] + 1
        ring_ok = (t - consumed[c] <= D) or cfg.bug == "no_ring_check"
        if ring_ok:
            j, half = (0, 0) if stage < 0 else divmod(stage, 2)
            w = members[j]
            slot = t % D
            seq, code, pay = cmd[w][slot]
            first, second = ("word", "payload") if cfg.bug == "cmd_before_payload" else ("payload", "word")
            step = first if half == 0 else second
            if step == "payload":
                ncmd = _set(cmd, w, _set(cmd[w], slot, (seq, code, nxt_item)))
            else:
                ncmd = _set(cmd, w, _set(cmd[w], slot, (t, TO_WORK, pay)))
            nstage = stage + 1 if stage >= 0 else 1
            if nstage == 2 * len(members):
                nhost = (nxt_item + 1, -1, _set(posted, c, t), consumed, exit_w, exit_stage)
            else:
                nhost = (nxt_item, nstage, posted, consumed, exit_w, exit_stage)
            yield ("post", (ncmd, status, workers, outputs, executed, nhost))

    # --- host: wait for (and consume) the oldest unconsumed ticket of any cluster.
    for c, members in enumerate(cfg.clusters):
        t = consumed[c] + 1
        if t > posted[c]:
            continue
        slot = t % D
        if all(status[w][slot] == (t, FROM_FINISHED) for w in members):
            item = _item_of(cfg, c, t)
            for w in members:
                if (item, w) not in outputs:
                    raise Violation(f"I4: completion of item {item} seen before output of worker {w}")
            nhost = (nxt_item, stage, posted, _set(consumed, c, t), exit_w, exit_stage)
            yield ("wait", (cmd, status, workers, outputs, executed, nhost))

    # --- host: once every item is consumed, post EXIT to each worker in turn.
    all_done = nxt_item == len(cfg.items) and all(consumed[c] == posted[c] for c in range(len(cfg.clusters)))
    if all_done and exit_w < cfg.n_workers:
        w = max(exit_w, 0)
        if w < cfg.n_workers:
            c = _cluster_of(cfg, w)
            t = posted[c] + 1
            slot = t % D
            seq, code, pay = cmd[w][slot]
            ncmd = _set(cmd, w, _set(cmd[w], slot, (t, TO_EXIT, -1)))
            nhost = (nxt_item, stage, posted, consumed, w + 1, exit_stage)
            yield ("exit", (ncmd, status, workers, outputs, executed, nhost))

    # --- workers
    for w, (done, phase, cur, exited, ahead) in enumerate(workers):
        if phase == 3:
            continue
        if phase == 0:   # poll the next slot; accept only the expected sequence number
            slot = (done + 1) % D
            if ahead is not None and (ahead[0] == done + 1 or cfg.bug == "ahead_no_seq"):
                # the snapshot taken during the previous item is the command (planted bug
                # "ahead_no_seq": used without checking its sequence number)
                seq, code, pay = ahead
                ok = True
            else:
                seq, code, pay = cmd[w][slot]
                # planted bug "no_seq": a lone code word without a sequence number, so any
                # WORK word in the slot looks new (the naive reading of Table 1).
                ok = seq == done + 1 or (cfg.bug == "no_seq" and code == TO_WORK and seq > 0)
            if not ok:
                continue
            if code == TO_EXIT:
                nw = _set(workers, w, (done + 1, 3, -1, 1, None))
                yield (f"w{w}exit", (cmd, status, nw, outputs, executed, host))
                continue
            nw = _set(workers, w, (done + 1, 1, pay, 0, None))
            nexec = executed + ((w, done + 1, pay),)
            yield (f"w{w}pick", (cmd, status, nw, outputs, nexec, host))
            continue
        if cfg.lookahead and D > 1 and ahead is None:   # look-ahead read during the item
            snap = cmd[w][(done + 1) % D]
            nw = _set(workers, w, (done, phase, cur, 0, snap))
            yield (f"w{w}ahead", (cmd, status, nw, outputs, executed, host))
        if phase == 1:   # execute: write the output (or, planted bug, publish first)
            if cfg.bug == "status_before_output":
                nst = _set(status, w, _set(status[w], done % D, (done, FROM_FINISHED)))
                nw = _set(workers, w, (done, 2, cur, 0, ahead))
                yield (f"w{w}pub", (cmd, nst, nw, outputs, executed, host))
            else:
                nw = _set(workers, w, (done, 2, cur, 0, ahead))
                yield (f"w{w}out", (cmd, status, nw, outputs | {(cur, w)}, executed, host))
        elif phase == 2:   # release: publish FINISHED (or, planted bug, write the output last)
            if cfg.bug == "status_before_output":
                nw = _set(workers, w, (done, 0, -1, 0, ahead))
                yield (f"w{w}out", (cmd, status, nw, outputs | {(cur, w)}, executed, host))
            else:
                nst = _set(status, w, _set(status[w], done % D, (done, FROM_FINISHED)))
                nw = _set(workers, w, (done, 0, -1, 0, ahead))
                yield (f"w{w}pub", (cmd, nst, nw, outputs, executed, host))


def _check_state(cfg, st):
    cmd, status, workers, outputs, executed, host = st
    seen = set()
    last = {}
    for (w, seq, item) in executed:
        if (w, seq) in seen:
            raise Violation(f"I1: worker {w} executed seq {seq} twice")
        seen.add((w, seq))
        if seq != last.get(w, 0) + 1:
            raise Violation(f"I2: worker {w} executed seq {seq} after {last.get(w, 0)}")
        last[w] = seq
        if item < 0 or item >= len(cfg.items):
            raise Violation(f"I1: worker {w} executed seq {seq} with a stale payload")
        c = cfg.items[item]
        if w not in cfg.clusters[c]:
            raise Violation(f"I3: item {item} of cluster {c} executed by worker {w}")
        if _ticket_of_item(cfg, item) != seq:
            raise Violation(f"I1: worker {w} seq {seq} carried item {item} (ticket mismatch)")


def _is_final(cfg, st):
    cmd, status, workers, outputs, executed, host = st
    return all(p == 3 for (_, p, _, _, _) in workers) and host[0] == len(cfg.items)


def check(cfg, max_states=2_000_000):
    """Explore every interleaving; raise Violation on the first broken property.
    Returns the number of reachable states."""
    init = _initial(cfg)
    seen = {init: None}
    stack = [init]
    succ = {}
    while stack:
        st = stack.pop()
        _check_state(cfg, st)
        nexts = [s for _, s in _steps(cfg, st)]
        succ[st] = nexts
        if not nexts and not _is_final(cfg, st):
            raise Violation("deadlock: no enabled step in a non-final state")
        for s in nexts:
            if s not in seen:
                seen[s] = None
                stack.append(s)
                if len(seen) > max_states:
                    raise RuntimeError("state space too large for this configuration")
    # Final state reachable from every state: backward reachability from final states.
    pred = {s: [] for s in succ}
    for s, ns in succ.items():
        for n in ns:
            pred[n].append(s)
    good = [s for s in succ if _is_final(cfg, s)]
    if not good:
        raise Violation("liveness: no final state is reachable")
    reach = set(good)
    frontier = list(good)
    while frontier:
        s = frontier.pop()
        for p in pred[s]:
            if p not in reach:
                reach.add(p)
                frontier.append(p)
    if len(reach) != len(succ):
        raise Violation("liveness: some reachable state cannot reach the final state")
    return len(succ)
