"""Point source convention for the nonhomogeneous terms.

The paper omits the nonhomogeneous vector terms of its splitting formulae (Sec.
II, opening paragraph).  The convention used here, identical for every scheme
and form:

* a sub-step that advances with the Cayley factor of operator X and half-span
  theta, written in original form as (I - theta X) u' = (I + theta Y) u + g,
  receives the vector g with a single nonzero entry at the Ez node of the source
  cell:  g = theta * f(t_k),  f(t) = amp * p(t),
  p(t) = exp(-((t - t0)/tau)^2) * sin(2 pi f0 (t - t0));
* t_k is the middle of the sub-step's nominal time interval
  (ADI, LOD1: n+1/4 and n+3/4; SS2: n+1/8, n+1/2, n+7/8; LOD2 main
  iteration: n+1/2 and n+1, in units of dt); LOD2 input/output processing has
  no source.

Over one full step the terms add up to dt * f for every scheme.  In the
fundamental forms the same g enters as described in ``fundamental``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class Source:
    i: int
    j: int
    k: int
    f0: float = 10e9
    tau: float = 0.1e-9
    t0: float = 0.4e-9
    amp: float = 1.0e10

    def pulse(self, t: float) -> float:
        x = (t - self.t0) / self.tau
        return math.exp(-x * x) * math.sin(2.0 * math.pi * self.f0 * (t - self.t0))

    def g(self, theta: float, t: float) -> float:
        """Entry of the nonhomogeneous vector at the Ez node of the source cell."""
        return theta * self.amp * self.pulse(t)
