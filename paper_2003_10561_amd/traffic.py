"""Algorithmic HBM bytes of one AT step (what the method must move per grid point).

Per point and step the low-storage RK3 reads and writes the state and its register:
stage 1 reads Q and writes Q and dQ (15 words), stage 2 reads Q and dQ and writes both (20),
stage 3 reads Q and dQ and writes Q (15) -> 50 words.  Each step publishes the two face layers
of every PE (u, v, w, T and the 5 face-normal fluxes: 9 words on a fraction
phi = 4 (1/ex + 1/ey + 1/ez) of the points).  A step whose faces are delayed reads 3 levels of those
9 words behind its delayed faces: the levels are the same for the three stages (only the
extrapolation weights differ, Sec. 2.1), so the method needs them once per step: 27 phi p_d words,
with p_d the fraction of (step, face) pairs whose delay is >= 1.  Halo re-reads of neighbouring
points are assumed to be served by on-chip caches and are not algorithmic.

`words_per_point_step_stage_reads` is the looser count that charges the delayed-level reads to
each of the three stages (81 phi p_d); it is reported beside the minimal one, never used for the
roofline fraction.
"""
from __future__ import annotations


def ghost_fraction(n, p, order: int = 4) -> float:
    """Fraction of points on published face layers: 2 M (1/ex + 1/ey + 1/ez), M = order / 2."""
    return sum(order * p[d] / n[d] for d in range(3))


def words_per_point_step(n, p, p_delayed: float, order: int = 4) -> float:
    """Minimal words per point-step of an RK3 step (delayed levels read once per step; the
    sixth-order scheme extrapolates from t_l = 4 levels instead of 3)."""
    phi = ghost_fraction(n, p, order)
    tl = order // 2 + 1
    return 50.0 + 9.0 * phi + 9.0 * tl * phi * p_delayed


def words_per_point_step_stage_reads(n, p, p_delayed: float) -> float:
    """The same with the delayed levels read again by each of the three stages."""
    phi = ghost_fraction(n, p)
    return 50.0 + 9.0 * phi + 3.0 * 27.0 * phi * p_delayed


def bytes_per_point_step(n, p, p_delayed: float, word: int) -> float:
    return word * words_per_point_step(n, p, p_delayed)


def ab2_words_per_point_step(n, p, p_delayed: float) -> float:
    """Second-order Adams-Bashforth (Sec. 2.2, Eq. time_ab): one stage per step reads Q and the
    stored dt f^{n-1} and writes Q and dt f^n (20 words), publishes the face layers (9 phi) and, on
    delayed faces, reads 3 levels of the 9 ghost words once (27 phi p_d)."""
    phi = ghost_fraction(n, p)
    return 20.0 + 9.0 * phi + 27.0 * phi * p_delayed


def paper_words_per_point_step(n, p, p_delayed: float, ab2: bool = False) -> float:
    """The paper's own discretisation (form 1): the RK3 state and register traffic (50 words; 20 for
    an Adams-Bashforth step), the publication of the five conserved variables on the face layers
    (5 phi) and, behind delayed faces, 3 levels of those 5 words read once per step (15 phi p_d).
    The gradients that the mixed derivatives differentiate again are not algorithmic traffic (a
    kernel could keep them on chip); this implementation writes and reads them (24 words a stage)."""
    phi = ghost_fraction(n, p)
    return (20.0 if ab2 else 50.0) + 5.0 * phi + 15.0 * phi * p_delayed


def delayed_fraction(table) -> float:
    """Fraction of (step, PE, face) entries with delay >= 1 in an int8 schedule table."""
    import numpy as np
    t = np.asarray(table)
    return float((t > 0).mean()) if t.size else 0.0
