"""How far a workload's photon histories move under last-bit rounding alone.

The oracle is run twice on the same photons: as built (no fused multiply-adds)
and perturbed, i.e. built with fused multiply-adds and run on the box
translated by four box widths (every position and cell face then rounds
differently).  Both runs compute the same method exactly; any history that
differs between them was turned by a rounding difference that some step of the
method amplified (local core-skipping makes x_crit depend on the distance to
the nearest face; aggressive core-skipping and long histories add more
branches).  The GPU computes in other units with other library functions, so
its histories may differ from the oracle's by about as much: parity tests take
their tolerance for diverging histories from this measured fraction instead of
a fixed guess.  Test infrastructure only.
"""
import math

import numpy as np

import oracle


def translated(grid, source, shift_widths=4.0):
    width = np.asarray(grid["box_max"], float) - np.asarray(grid["box_min"], float)
    off = shift_widths * width
    g = dict(grid, box_min=np.asarray(grid["box_min"], float) + off,
             box_max=np.asarray(grid["box_max"], float) + off)
    s = dict(source, pos=np.asarray(source["pos"], float).reshape(-1, 3) + off)
    return g, s


def self_divergence(grid, source, params, id_begin=0, id_end=None, threads=None):
    """Fraction of photons in [id_begin, id_end) whose scattering count or
    outcome differs between the plain and the perturbed oracle."""
    a = oracle.run(grid, source, params, id_begin=id_begin, id_end=id_end, records=True,
                   threads=threads)["records"]
    g, s = translated(grid, source)
    b = oracle.run(g, s, params, id_begin=id_begin, id_end=id_end, records=True,
                   threads=threads, variant="fma")["records"]
    same = (a["nscat"] == b["nscat"]) & (a["status"] == b["status"])
    return 1.0 - float(same.mean())


def flip_tolerance(self_div, n, floor=0.005):
    """Diverging-history fraction a GPU run may show: the oracle's own
    divergence under the perturbation, half again for the GPU's further
    differences (units, library functions), three binomial standard errors,
    and a floor for workloads the perturbation leaves untouched."""
    se = math.sqrt(max(self_div * (1.0 - self_div), 1.0 / n) / n)
    return min(1.0, floor + 1.5 * self_div + 3.0 * se)
