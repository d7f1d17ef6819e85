"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module holds no harmonic-summing arithmetic: it only draws filter-output
planes (FOPs) of the paper's shape (N_temp templates x N_chan bins of fp32
power, Sec. III and its specification table: 85 x 2^21, 8 planes) and the
threshold arrays.  The real SKA FOPs are not available; these stand in.

Noise: x = (a^2 + b^2) / 2 with a, b ~ N(0, 1) iid, i.e. |complex N(0,1)|^2/2,
which is Exponential(1).  Signals: a fundamental at template z0, bin f0 with
power P0 adds P0/n at template n*z0, bin n*f0 for harmonics n = 1..n_h
(additive).  Thresholds: T_k = k + 6*sqrt(k) for every row, evaluated in fp64
and rounded once to fp32.

Draws use torch generators (on the device where the plane is made) and numpy
generators for the few signal parameters, so every input is a function of
its seed.
"""
import math

import numpy as np
import torch

# Workload shapes (rows, bins, planes) and seeds.
TINY = dict(name="tiny", n_temp=21, n_chan=1 << 16, n_hp=8, seed=1)
SKA = dict(name="ska", n_temp=85, n_chan=1 << 21, n_hp=8, seed=2)
BATCHED = dict(name="batched", n_fops=512, n_temp=85, lengths=(1 << 19, 1 << 20, 1 << 21),
               n_hp=16, seed=3)
PRECISION = dict(name="precision", n_fops=128, n_temp=85, n_chan=1 << 21, n_hp=8, seed=4,
                 input_scale=0.125)
DIFF = dict(name="diff", n_fops=16, n_temp=85, n_chan=1 << 20, n_hp=8, seed=5, tau=0.5)


def thresholds(n_hp, n_temp):
    """[H][T] fp32 thresholds, T_k = k + 6 sqrt(k) on every row."""
    t = np.array([k + 6.0 * math.sqrt(k) for k in range(1, n_hp + 1)], dtype=np.float64)
    return np.repeat(t.astype(np.float32)[:, None], n_temp, axis=1)


def noise(n_temp, n_chan, seed, device="cpu", ld=None, dtype=torch.float32):
    """Exp(1) power plane [T][ld] (columns >= n_chan are zero), seeded."""
    ld = n_chan if ld is None else ld
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.zeros((n_temp, ld), dtype=torch.float32, device=device)
    for r in range(n_temp):
        ab = torch.randn((2, n_chan), generator=g, device=device, dtype=torch.float32)
        out[r, :n_chan] = (ab[0] * ab[0] + ab[1] * ab[1]) * 0.5
    return out if dtype == torch.float32 else out.to(dtype)


def draw_signals(n_temp, n_chan, n_hp, count, seed, p0_range=(8.0, 40.0), max_harm=None):
    """Random signals (z0, f0, P0, n_h) whose harmonic cells do not overlap."""
    rng = np.random.default_rng(int(seed) + 7919)
    c = n_temp // 2
    max_harm = n_hp if max_harm is None else max_harm
    used = set()
    sigs = []
    tries = 0
    while len(sigs) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place signals")
        nh = int(rng.integers(1, max_harm + 1))
        zmax = c // nh
        z0 = int(rng.integers(-zmax, zmax + 1))
        fhi = (n_chan - 1) // nh
        flo = n_hp + 1
        if fhi < flo:
            continue
        f0 = int(rng.integers(flo, fhi + 1))
        p0 = float(rng.uniform(*p0_range))
        cells = [(n * z0, n * f0) for n in range(1, nh + 1)]
        if any(cell in used for cell in cells):
            continue
        used.update(cells)
        sigs.append((z0, f0, p0, nh))
    return sigs


def tiny_signals():
    """The three signals of the tiny plane: z0 in {0, +1, -1}, P0 = 20, 8 harmonics."""
    rng = np.random.default_rng(TINY["seed"] + 104729)
    f0s = rng.integers(9, 8192, size=3)
    return [(0, int(f0s[0]), 20.0, 8), (1, int(f0s[1]), 20.0, 8), (-1, int(f0s[2]), 20.0, 8)]


def inject(fop, signals):
    """Add P0/n at (row n*z0 + T//2, bin n*f0) for each signal, in place."""
    c = fop.shape[0] // 2
    for z0, f0, p0, nh in signals:
        for n in range(1, nh + 1):
            fop[n * z0 + c, n * f0] += p0 / n
    return fop


def make_tiny(device="cpu"):
    fop = noise(TINY["n_temp"], TINY["n_chan"], TINY["seed"], device)
    return inject(fop, tiny_signals())


def make_ska(device="cpu", seed=None):
    s = SKA["seed"] if seed is None else seed
    fop = noise(SKA["n_temp"], SKA["n_chan"], s, device)
    return inject(fop, draw_signals(SKA["n_temp"], SKA["n_chan"], SKA["n_hp"], 50, s))


def batched_lengths(n_fops=None, seed=None):
    """Bin count of each FOP of the batched workload, drawn from {2^19, 2^20, 2^21}."""
    n = BATCHED["n_fops"] if n_fops is None else n_fops
    s = BATCHED["seed"] if seed is None else seed
    rng = np.random.default_rng(s)
    return [int(x) for x in rng.choice(np.array(BATCHED["lengths"]), size=n)]


def make_batched_fop(f, n_chan, device="cpu", ld=None):
    """FOP f of the batched workload (seed 3*10^6 + f, 0-5 signals)."""
    s = 3 * 10 ** 6 + f
    fop = noise(BATCHED["n_temp"], n_chan, s, device, ld=ld)
    nsig = int(np.random.default_rng(s).integers(0, 6))
    return inject(fop, draw_signals(BATCHED["n_temp"], n_chan, BATCHED["n_hp"], nsig, s))


def make_precision_fop(f, device="cpu"):
    """FOP f of the precision workload in fp32 (seed 4*10^6 + f, 50 signals)."""
    s = 4 * 10 ** 6 + f
    fop = noise(PRECISION["n_temp"], PRECISION["n_chan"], s, device)
    return inject(fop, draw_signals(PRECISION["n_temp"], PRECISION["n_chan"],
                                    PRECISION["n_hp"], 50, s))


def make_diff_fop(f, device="cpu", n_chan=None):
    """FOP f of the differentiation workload (seed 5*10^6 + f, 5 signals)."""
    s = 5 * 10 ** 6 + f
    n = DIFF["n_chan"] if n_chan is None else n_chan
    fop = noise(DIFF["n_temp"], n, s, device)
    return inject(fop, draw_signals(DIFF["n_temp"], n, DIFF["n_hp"], 5, s))


def quantize(fop, dtype, scale):
    """Storage copy of x*scale in fp16/bf16 (round to nearest even)."""
    return (fop * scale).to(dtype)
