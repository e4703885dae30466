"""Per-sample random inputs, oracle side (test infrastructure only).

The random field of the workloads: the log wave speed g = log c is piecewise
constant on a block grid with i.i.d. N(0, sigma^2) values, kappa = c^2 =
exp(2 g) enters the stiffness (Sec. 2.1 / 3.1), and the initial Gaussian pulse
has a uniformly distributed centre.  Each sample omega^(i,l) of level l is
drawn from its own counter-based stream so that the fine and the coarse solve
of a difference Delta Q_l use the same omega (Sec. 2.2) and samples of
different levels are independent.

Stream layout (a reading; the paper fixes none):
  Philox4x64-10, key = (seed, 0), counter = (j, i, l, purpose),
  purpose 0 = field normals, 1 = pulse centre; block j yields 4 words.
  uniform u = ((x >> 12) + 0.5) * 2^-52  in (0, 1)
  Box-Muller on consecutive uniforms: r = sqrt(-2 log u_a), t = 2 pi u_b,
  (r cos t, r sin t).
  n_steps = ceil(T c_max / (cfl h)), dt = T / n_steps, c_max = max_b exp(g_b).

Philox itself comes from numpy.random.Philox (an implementation independent of
the library's); scalar math uses Python's ``math`` module.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MASK64 = (1 << 64) - 1


def philox_block(seed: int, ctr) -> list:
    """The four 64-bit output words of Philox4x64-10 at counter ``ctr`` (4 words)
    and key (seed, 0).  numpy's generator increments its counter before every
    block, so it is started one below the wanted counter."""
    c = sum((int(w) & MASK64) << (64 * k) for k, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    cw = np.array([(c >> (64 * k)) & MASK64 for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=cw, key=np.array([seed & MASK64, 0], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def philox_block_key(key, ctr) -> list:
    """Philox4x64-10 with an explicit 2-word key (used for known-answer tests)."""
    c = sum((int(w) & MASK64) << (64 * k) for k, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    cw = np.array([(c >> (64 * k)) & MASK64 for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=cw, key=np.array([k & MASK64 for k in key], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def to_uniform(x: int) -> float:
    return (float(x >> 12) + 0.5) * 2.0 ** -52


def uniforms(seed: int, i: int, level: int, purpose: int, n: int) -> list:
    out = []
    j = 0
    while len(out) < n:
        out += [to_uniform(w) for w in philox_block(seed, (j, i, level, purpose))]
        j += 1
    return out[:n]


@dataclass
class SampleRule:
    n_blocks: int = 16
    sigma: float = 0.25
    pulse_box: tuple = (0.2, 0.4, 0.2, 0.4)   # x_lo, x_hi, y_lo, y_hi
    T: float = 1.0
    cfl: float = 0.2


@dataclass
class Sample:
    g: list            # [n_blocks] log wave speed per block
    kappa: list        # [n_blocks] c^2 = exp(2 g)
    x0: tuple          # pulse centre
    c_max: float


def draw(seed: int, level: int, i: int, rule: SampleRule) -> Sample:
    nb = rule.n_blocks
    if nb % 2:
        raise ValueError("n_blocks must be even (Box-Muller pairs)")
    u = uniforms(seed, i, level, 0, nb)
    z = []
    for k in range(0, nb, 2):
        r = math.sqrt(-2.0 * math.log(u[k]))
        t = (2.0 * math.pi) * u[k + 1]
        z += [r * math.cos(t), r * math.sin(t)]
    g = [rule.sigma * zk for zk in z]
    kappa = [math.exp(2.0 * gk) for gk in g]
    c_max = max(math.exp(gk) for gk in g)
    up = uniforms(seed, i, level, 1, 2)
    bx0, bx1, by0, by1 = rule.pulse_box
    x0 = (bx0 + (bx1 - bx0) * up[0], by0 + (by1 - by0) * up[1])
    return Sample(g=g, kappa=kappa, x0=x0, c_max=c_max)


def steps_for(sample: Sample, rule: SampleRule, h: float):
    """n_steps = ceil(T c_max / (cfl h)), dt = T / n_steps on a mesh of base spacing h."""
    n = int(math.ceil((rule.T * sample.c_max) / (rule.cfl * h)))
    return n, rule.T / n
