"""Closed forms used as pins.

Scalar time-invariant problem (nx = nu = 1, S = 0): the fixed point of the
Riccati recursion (eq. riccati-recursion-P) solves
    b^2 P^2 + (r (1 - a^2) - q b^2) P - q r = 0,
whose positive root is the stabilising solution of the discrete algebraic
Riccati equation.
"""
from __future__ import annotations

import math


def scalar_dare(a, b, q, r):
    c = r * (1.0 - a * a) - q * b * b
    return (-c + math.sqrt(c * c + 4.0 * b * b * q * r)) / (2.0 * b * b)
