"""Width-update rule over time steps (Sec. II.D, the update algorithm).

Test infrastructure: see the package docstring.

The rule keeps a p-value threshold ``p_th``, the width in use ``h_opt`` and
a target width ``h_target``. After each push the positions' Anderson-Darling
p-value ``p`` is compared with it:

* p above twice the significance threshold (0.01): the positions look
  uniform, so only the threshold is reset to twice the significance level;
* otherwise, p below half of ``p_th``: the distribution has moved enough, so
  the CV objective is minimised again for a new target and ``p_th = p``;
* in every step the width relaxes towards the target at rate 0.05:
  ``h_opt <- rate h_target + (1 - rate) h_opt``.

The rule relaxes the width h; the concentration follows from
``kappa = (L/(2 pi h))^2``.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Callable, Tuple

THRESHOLD = 0.01
ADJUST_RATE = 0.05


@dataclass(frozen=True)
class UpdateState:
    p_th: float
    h_opt: float
    h_target: float


def initial_state(h0: float, threshold: float = THRESHOLD) -> UpdateState:
    """State after the CV solve at t = 0: both widths at its optimum and
    ``p_th = 2 * threshold``."""
    return UpdateState(2.0 * threshold, float(h0), float(h0))


def step(state: UpdateState, p: float, solve_width: Callable[[], float],
         threshold: float = THRESHOLD, rate: float = ADJUST_RATE) -> Tuple[UpdateState, bool]:
    """Apply one step of the rule; ``solve_width()`` runs the CV minimisation
    and is called only when the rule fires. Returns ``(new_state, fired)``."""
    fired = False
    s = state
    if p > 2.0 * threshold:
        s = replace(s, p_th=2.0 * threshold)
    elif p < 0.5 * s.p_th:
        s = replace(s, h_target=float(solve_width()), p_th=float(p))
        fired = True
    s = replace(s, h_opt=rate * s.h_target + (1.0 - rate) * s.h_opt)
    return s, fired
