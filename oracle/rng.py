"""Candidate sampling and stage schedule for the oracle (test infrastructure only).

Section 4 ("Sparse primal optimization") says that each basis-selection step draws a small random subset
of the training set and scores it, and that re-optimisation happens after "a certain number" of additions.
It fixes neither the subset size, the random stream, nor the stage sizes. The readings taken here:

* kappa = 59 candidates per step (the best of 59 uniform draws lies in the top 5% with probability
  1 - 0.95^59 > 0.95).
* Random stream: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), one counter stream per step.
  Step t (0-based index of the addition step, counted over the whole run) starts from state
  ``seed XOR ((t * 2^32 + 1) * GOLDEN mod 2^64)``. Each draw adds GOLDEN to the state and mixes it with the
  published finaliser (shifts 30, 27, 31; multipliers 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB).
  Section 4 draws a fresh random subset at every step, so the streams of different steps must not overlap:
  a step makes at most 64 kappa draws, far fewer than the 2^32 states between the starts of consecutive steps
  (with ``(t + 1) * GOLDEN`` instead, seed 0 would give step t + 1 the draws of step t shifted by one).
* Index: ``((z >> 32) * n) >> 32`` (the high 32 bits scaled to [0, n)).
* Rejection: a draw is rejected if it repeats an index already accepted in this step, or if its row
  is blocked (it is a basis member, or an exact duplicate of one, as J stood at the start of the
  stage). Drawing stops after kappa accepted indices or 64 * kappa attempts, whichever comes first.
* Stage size: c_s = min(J_max - |J|, max(1, min(cap, floor(growth * |J|)))) with growth = 0.25 and
  cap = 256.
"""

from __future__ import annotations

import math

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_stream(state: int, count: int) -> list[int]:
    """``count`` successive SplitMix64 outputs from ``state`` (state is advanced before each output)."""
    out = []
    for _ in range(count):
        state = (state + GOLDEN) & MASK64
        out.append(_mix(state))
    return out


def step_state(seed: int, t: int) -> int:
    return (seed ^ ((((t << 32) + 1) * GOLDEN) & MASK64)) & MASK64


def scaled_index(z: int, n: int) -> int:
    return ((z >> 32) * n) >> 32


def draw_candidates(seed: int, t: int, n: int, kappa: int, blocked) -> list[int]:
    """Candidate indices for addition step ``t``; ``blocked(i)`` says whether row i may not be drawn."""
    state = step_state(seed, t)
    chosen: list[int] = []
    taken = set()
    for _ in range(64 * kappa):
        if len(chosen) == kappa:
            break
        state = (state + GOLDEN) & MASK64
        i = scaled_index(_mix(state), n)
        if i in taken or blocked(i):
            continue
        taken.add(i)
        chosen.append(i)
    return chosen


def stage_size(J_size: int, J_max: int, growth: float = 0.25, cap: int = 256) -> int:
    """Number of additions before the next re-optimisation."""
    return min(J_max - J_size, max(1, min(cap, int(math.floor(growth * J_size)))))
