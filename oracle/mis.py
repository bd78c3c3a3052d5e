"""Metropolis independence chain over TN proposals (oracle side, float64).

Test infrastructure only: nothing in the product path imports this module.

Eq. (10) of section 2.3: a candidate s' drawn from q replaces the current
state s with probability min[1, q(s) P(s') / (q(s') P(s))].  In logs, with
the current state x and candidate k,

    delta = (log q_x - log q_k) + beta * (E_x - E_k),

each operation rounded separately (no fused multiply-add), and the candidate
is accepted iff delta >= 0 or u_k < exp(delta).

Readings (the paper gives no code for this step): one chain per instance
walks that instance's proposals in index order; on the very first call the
first proposal initialises the chain and is not counted as a trial; the chain
state (current log q, energy, global index, accepted and trial counts)
carries over between calls; u_k is Philox4x32-10 with counter
(global proposal index, 0, instance, 1).

Pins (tests/test_oracle_mis.py): in the exact regime every trial is
accepted; at truncated chi the histogram of chain states matches the
brute-force Boltzmann law (chi-squared) while the raw proposals do not.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox


class Chain:
    """Per-instance chain state."""

    def __init__(self):
        self.initialised = False
        self.cur_logq = 0.0
        self.cur_E = 0.0
        self.cur_index = -1
        self.n_acc = 0
        self.n_trials = 0


def accept(logq, E, beta, chain: Chain, seed: int, instance: int, step_offset: int):
    """Run one instance's chain over len(logq) proposals.

    Returns (accepted uint8 (n,), state index int64 (n,)): whether each
    proposal was accepted, and the global index of the chain state after it.
    """
    logq = np.asarray(logq, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    n = logq.shape[0]
    acc = np.zeros(n, dtype=np.uint8)
    idx = np.zeros(n, dtype=np.int64)
    beta = float(beta)
    for k in range(n):
        g = step_offset + k
        if not chain.initialised:
            chain.initialised = True
            chain.cur_logq, chain.cur_E, chain.cur_index = float(logq[k]), float(E[k]), g
            acc[k] = 1
            idx[k] = g
            continue
        d_logq = chain.cur_logq - float(logq[k])
        d_E = chain.cur_E - float(E[k])
        delta = d_logq + beta * d_E          # Python floats: one rounding per op
        u = float(philox.uniform(seed, g, 0, instance, philox.STREAM_ACCEPT))
        ok = delta >= 0.0 or u < math.exp(delta)
        chain.n_trials += 1
        if ok:
            chain.n_acc += 1
            chain.cur_logq, chain.cur_E, chain.cur_index = float(logq[k]), float(E[k]), g
            acc[k] = 1
        idx[k] = chain.cur_index
    return acc, idx
