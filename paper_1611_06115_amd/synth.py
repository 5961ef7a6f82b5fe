"""Seeded synthetic inputs: genome-shaped texts, IUPAC patterns, planted sites.

Input generation only -- nothing here encodes, scores or counts; texts are
ASCII letters and patterns are IUPAC strings.  The tests, the benchmark and
the oracle's inputs all come from here.

Randomness is counter based (SplitMix64 output function applied to
``key + G*(i+1)``, Steele, Lea & Flood 2014) and addressed by
(seed, stream, index), so every piece regenerates identically anywhere.
Base seed 161106115; workload c uses seed 161106115 + c; streams are
0 = text, 1 = patterns, 2 = plants, 3 = query pool, 4 = arrivals.

Workloads (sizes and shapes of the paper's setting, Sect. 3: a long human
chromosome and long patterns cut from it; no real sequence is used):

* ``small``    1e6 uniform bases; m = 32 (24 singletons + 8 multi-base
               classes); 64 planted copies with d in {0,1,2,3}; k in {0, 2}.
* ``long_m``   64e6 i.i.d. bases at GC 41%; m = 1024 and 4096 (90% singletons,
               the rest 2-3-base classes); 32 plants per pattern, d in
               {0, 4, 16, 17}; k in {0, 4, 16}.
* ``genome``   3.1e9 bases from an order-3 Markov chain at GC 41%; m = 256
               with 20% 2-3-base classes; 64 plants, d in 0..5; k = 4.
* ``batched``  256e6 i.i.d. bases at GC 41%; 4096 patterns, m ~ U{16..2048},
               class density ~ U[0, 0.3], k ~ U{0..8}; 2 plants per pattern.
* ``served``   the genome text; a pool of queries with m log-uniform over
               [20, 5000], k ~ U{0..10}, density ~ U[0, 0.3], each planted
               once; Poisson arrivals.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

SEED0 = 161106115
STREAM_TEXT, STREAM_PATTERNS, STREAM_PLANTS, STREAM_POOL, STREAM_ARRIVALS = range(5)
GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

# IUPAC one-letter classes -> member bases (the standard nomenclature).
IUPAC_MEMBERS = {
    "A": "A", "C": "C", "G": "G", "T": "T",
    "M": "AC", "R": "AG", "W": "AT", "S": "CG", "Y": "CT", "K": "GT",
    "V": "ACG", "H": "ACT", "D": "AGT", "B": "CGT", "N": "ACGT", "-": "",
}
SINGLETONS = "ACGT"
TWO_THREE = "MRWSYKVHDB"            # the 10 classes of 2 or 3 bases
MULTI = TWO_THREE + "N"             # the 11 classes of 2 or more bases
GC41 = (0.295, 0.205, 0.205, 0.295)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "synth.c")
_LIB = os.path.join(_HERE, "libpmsynth.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.pms_key.argtypes = [u64, u64]
        lib.pms_key.restype = u64
        lib.pms_draw.argtypes = [u64, u64]
        lib.pms_draw.restype = u64
        lib.pms_iid.argtypes = [p, u64, u64, p, ctypes.c_int]
        lib.pms_iid.restype = ctypes.c_int
        lib.pms_markov3.argtypes = [p, u64, u64, p, p, u64, ctypes.c_int]
        lib.pms_markov3.restype = ctypes.c_int
        _lib = lib
    return _lib


def gen_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --- counter-based draws ----------------------------------------------------

def _mix64(z):
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & MASK64
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB & MASK64
    return z ^ (z >> 31)


def key(seed: int, stream: int) -> int:
    return _mix64((seed * GOLDEN + stream + 1) & MASK64)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


class Draws:
    """Counter-based stream: value i = mix64(key + G*(i+1)); sub-streams by tag."""

    def __init__(self, k: int):
        self.key = k & MASK64

    def sub(self, tag: int) -> "Draws":
        return Draws(_mix64((self.key ^ (GOLDEN * (tag + 1))) & MASK64))

    def u64(self, i: int = 0, count: int | None = None):
        if count is None:
            return _mix64((self.key + GOLDEN * (i + 1)) & MASK64)
        idx = np.arange(i, i + count, dtype=np.uint64)
        with np.errstate(over="ignore"):
            return _mix64_np(np.uint64(self.key) + np.uint64(GOLDEN) * (idx + np.uint64(1)))

    def uniform(self, i: int = 0, count: int | None = None):
        v = self.u64(i, count)
        if count is None:
            return (v >> 11) * (1.0 / (1 << 53))
        return (v >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))

    def below(self, n: int, i: int = 0, count: int | None = None):
        u = self.uniform(i, count)
        if count is None:
            return min(int(u * n), n - 1)
        return np.minimum((u * n).astype(np.int64), n - 1)

    def subset(self, n: int, size: int) -> np.ndarray:
        """A uniformly random subset of exactly `size` indices of range(n)."""
        order = np.argsort(self.u64(0, n), kind="stable")
        return np.sort(order[:size])


# --- texts ------------------------------------------------------------------

def _thresholds(probs) -> np.ndarray:
    c = np.cumsum(np.asarray(probs, dtype=np.float64))[:3]
    return np.clip(np.rint(c * 65536.0), 0, 65535).astype(np.uint16)


def iid_text(n: int, seed: int, probs=(0.25, 0.25, 0.25, 0.25), threads: int | None = None,
             out: np.ndarray | None = None) -> np.ndarray:
    """n i.i.d. bases (ASCII) with P(A), P(C), P(G), P(T) = probs."""
    buf = np.empty(n, dtype=np.uint8) if out is None else out
    thr = _thresholds(probs)
    rc = _load().pms_iid(buf.ctypes.data, n, key(seed, STREAM_TEXT), thr.ctypes.data,
                         threads or gen_threads())
    if rc != 0:
        raise RuntimeError("text generation failed")
    return buf


@dataclass
class MarkovModel:
    rows: np.ndarray        # (64, 4) transition probabilities, ctx = b3<<4|b2<<2|b1
    stationary: np.ndarray  # (64,) stationary context law
    gc: float
    lam: float


def _stationary(rows: np.ndarray) -> np.ndarray:
    t = np.zeros((64, 64))
    for ctx in range(64):
        for b in range(4):
            t[ctx, ((ctx << 2) | b) & 63] += rows[ctx, b]
    pi = np.full(64, 1.0 / 64)
    for _ in range(10000):
        nxt = pi @ t
        if np.abs(nxt - pi).max() < 1e-15:
            pi = nxt
            break
        pi = nxt
    return pi / pi.sum()


def markov_model(seed: int, gc_target: float = 0.41) -> MarkovModel:
    """Order-3 chain: row weights w_b ~ U(0.5, 1.5) * prior(0.295, 0.205, 0.205,
    0.295); C and G weights scaled by lambda, chosen by bisection so that the
    stationary GC fraction is gc_target (to 1e-6)."""
    d = Draws(key(seed, STREAM_TEXT)).sub(0xC0FFEE)
    w = (0.5 + d.uniform(0, 256)).reshape(64, 4) * np.asarray(GC41)

    def model(lam):
        x = w.copy()
        x[:, 1:3] *= lam
        rows = x / x.sum(axis=1, keepdims=True)
        pi = _stationary(rows)
        gc = float((pi[:, None] * rows)[:, 1:3].sum())
        return rows, pi, gc

    lo, hi = -6.0, 6.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        _, _, gc = model(math.exp(mid))
        if gc < gc_target:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-12:
            break
    lam = math.exp(0.5 * (lo + hi))
    rows, pi, gc = model(lam)
    return MarkovModel(rows, pi, gc, lam)


def markov_text(n: int, seed: int, model: MarkovModel | None = None, chunk: int = 1 << 24,
                threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    model = model or markov_model(seed)
    thr = np.concatenate([_thresholds(r) for r in model.rows]).astype(np.uint16)
    start = np.clip(np.rint(np.cumsum(model.stationary)[:63] * 65536.0), 0, 65535).astype(np.uint16)
    buf = np.empty(n, dtype=np.uint8) if out is None else out
    rc = _load().pms_markov3(buf.ctypes.data, n, key(seed, STREAM_TEXT), thr.ctypes.data,
                             start.ctypes.data, chunk, threads or gen_threads())
    if rc != 0:
        raise RuntimeError("text generation failed")
    return buf


# --- patterns and plants ----------------------------------------------------

def random_pattern(d: Draws, m: int, n_class: int, classes: str = TWO_THREE) -> str:
    """m positions; exactly n_class of them (a random subset) hold a class
    drawn uniformly from `classes`, the others a uniform singleton base."""
    letters = np.frombuffer(SINGLETONS.encode(), dtype=np.uint8)[d.sub(2).below(4, 0, m)]
    if n_class:
        where = d.sub(1).subset(m, n_class)
        cls = d.sub(3).below(len(classes), 0, m)
        letters[where] = np.frombuffer(classes.encode(), dtype=np.uint8)[cls[where]]
    return letters.tobytes().decode("ascii")


def plant(text: np.ndarray, pos: int, pattern: str, dist: int, d: Draws) -> int:
    """Write a copy of `pattern` at text[pos:pos+m]: each position gets a
    uniform member of its class, then exactly `dist` positions (a random
    subset of those whose class is not N) get a base outside their class.
    Returns the number of positions altered (dist, or fewer when the pattern
    has fewer than dist eligible positions)."""
    m = len(pattern)
    pat = np.frombuffer(pattern.upper().encode("ascii"), dtype=np.uint8)
    pick = d.sub(1).u64(0, m)
    out = np.empty(m, dtype=np.uint8)
    for ch in np.unique(pat).tolist():
        mem = np.frombuffer((IUPAC_MEMBERS[chr(ch)] or "ACGT").encode(), dtype=np.uint8)
        sel = np.nonzero(pat == ch)[0]
        out[sel] = mem[(pick[sel] % np.uint64(mem.size)).astype(np.int64)]
    eligible = np.nonzero(pat != ord("N"))[0]
    dist = min(dist, int(eligible.size))
    if dist:
        chosen = eligible[d.sub(2).subset(int(eligible.size), dist)]
        alt = d.sub(3).u64(0, dist)
        for r, j in enumerate(chosen.tolist()):
            others = [b for b in "ACGT" if b not in IUPAC_MEMBERS[chr(pat[j])]]
            out[j] = ord(others[int(alt[r] % np.uint64(len(others)))])
    text[pos:pos + m] = out
    return dist


def plant_slots(n: int, m_max: int, count: int, d: Draws) -> list[int]:
    """`count` non-overlapping plant positions: one per equal text segment, at a
    random offset inside it (segments must hold m_max bases)."""
    seg = n // count
    if seg < m_max:
        raise ValueError("text too short for the requested plants")
    offs = d.below(seg - m_max + 1, 0, count)
    return [i * seg + int(offs[i]) for i in range(count)]


@dataclass
class Workload:
    name: str
    seed: int
    n: int
    text: np.ndarray
    patterns: list = field(default_factory=list)   # IUPAC strings
    ks: list = field(default_factory=list)         # k per pattern (or per run)
    plants: list = field(default_factory=list)     # (pattern index, pos, d)


def small(n: int = 1_000_000, m: int = 32, n_class: int = 8, n_plants: int = 64) -> Workload:
    seed = SEED0 + 0
    text = iid_text(n, seed)
    pat = random_pattern(Draws(key(seed, STREAM_PATTERNS)), m, n_class, MULTI)
    pd = Draws(key(seed, STREAM_PLANTS))
    slots = plant_slots(n, m, n_plants, pd.sub(0))
    plants = []
    for i, pos in enumerate(slots):
        dist = i % 4
        dist = plant(text, pos, pat, dist, pd.sub(100 + i))
        plants.append((0, pos, dist))
    return Workload("small", seed, n, text, [pat], [0, 2], plants)


def long_m(n: int = 64_000_000, ms=(1024, 4096), n_plants: int = 32) -> Workload:
    seed = SEED0 + 1
    text = iid_text(n, seed, GC41)
    pats = []
    pd = Draws(key(seed, STREAM_PLANTS))
    plants = []
    for pi, m in enumerate(ms):
        n_class = m - int(round(0.9 * m))
        pats.append(random_pattern(Draws(key(seed, STREAM_PATTERNS)).sub(pi), m, n_class))
    slots = plant_slots(n, max(ms), n_plants * len(ms), pd.sub(0))
    dists = (0, 4, 16, 17)
    for s, pos in enumerate(slots):
        pi = s % len(ms)
        dist = dists[(s // len(ms)) % 4]
        dist = plant(text, pos, pats[pi], dist, pd.sub(100 + s))
        plants.append((pi, pos, dist))
    return Workload("long_m", seed, n, text, pats, [0, 4, 16], plants)


def genome_pattern(seed: int = SEED0 + 2, m: int = 256, density: float = 0.2) -> str:
    return random_pattern(Draws(key(seed, STREAM_PATTERNS)), m, int(round(density * m)))


def genome(n: int = 3_100_000_000, m: int = 256, n_plants: int = 64,
           text: np.ndarray | None = None) -> Workload:
    seed = SEED0 + 2
    text = markov_text(n, seed, out=text)
    pat = genome_pattern(seed, m)
    pd = Draws(key(seed, STREAM_PLANTS))
    plants = []
    for i, pos in enumerate(plant_slots(n, m, n_plants, pd.sub(0))):
        dist = plant(text, pos, pat, i % 6, pd.sub(100 + i))
        plants.append((0, pos, dist))
    return Workload("genome", seed, n, text, [pat], [4], plants)


# The m-scaling experiment of Sect. 3 (Tables 5-7): chromosome 2's length
# and, per pattern length, the first printed location of each table row
# (1-based; Table 5 row 1 prints its range in reverse order, and its lower
# end is taken).
CHR2_LEN = 243_199_373
MSCALE_SITES = {
    500: (150967401, 52803498, 8749475, 234748299, 90472976),
    10000: (234097372, 33957613, 7034775, 115305600, 199419896),
    100000: (234097372, 33957613, 7034775, 115305600, 199419896),
}


def mscale(n: int = CHR2_LEN) -> Workload:
    """A chromosome-2-sized order-3 Markov text (GC 41%) and exact copies of
    it of m = 500, 10 000 and 100 000, cut at the five sites per length that
    Tables 5-7 list (0-based start = location - 1, moved left when the text
    is shorter than the chromosome); plants are the cut sites (d = 0)."""
    seed = SEED0 + 6
    text = markov_text(n, seed)
    pats, plants = [], []
    for m, sites in MSCALE_SITES.items():
        if m > n:
            continue
        for site in sites:
            p0 = min(site - 1, n - m)
            pats.append(text[p0:p0 + m].tobytes().decode())
            plants.append((len(pats) - 1, p0, 0))
    return Workload("mscale", seed, n, text, pats, [0] * len(pats), plants)


def batched_patterns(count: int = 4096, seed: int = SEED0 + 3, m_lo: int = 16,
                     m_hi: int = 2048, k_hi: int = 8, dens_hi: float = 0.3):
    d = Draws(key(seed, STREAM_PATTERNS))
    ms = m_lo + d.sub(1).below(m_hi - m_lo + 1, 0, count)
    dens = d.sub(2).uniform(0, count) * dens_hi
    ks = d.sub(3).below(k_hi + 1, 0, count)
    pats = [random_pattern(d.sub(1000 + i), int(ms[i]), int(round(dens[i] * ms[i])))
            for i in range(count)]
    return pats, [int(x) for x in ks]


def batched(n: int = 256_000_000, count: int = 4096, m_hi: int = 2048) -> Workload:
    seed = SEED0 + 3
    text = iid_text(n, seed, GC41)
    pats, ks = batched_patterns(count, seed, m_hi=m_hi)
    pd = Draws(key(seed, STREAM_PLANTS))
    plants = []
    slots = plant_slots(n, max(len(p) for p in pats), 2 * count, pd.sub(0))
    for s, pos in enumerate(slots):
        pi = s // 2
        dist = 0 if s % 2 == 0 else ks[pi]
        dist = plant(text, pos, pats[pi], dist, pd.sub(100 + s))
        plants.append((pi, pos, dist))
    return Workload("batched", seed, n, text, pats, ks, plants)


def query_pool(count: int = 20000, seed: int = SEED0 + 4, m_lo: int = 20, m_hi: int = 5000,
               k_hi: int = 10, dens_hi: float = 0.3):
    d = Draws(key(seed, STREAM_POOL))
    u = d.sub(1).uniform(0, count)
    ms = np.rint(np.exp(math.log(m_lo) + u * (math.log(m_hi) - math.log(m_lo)))).astype(np.int64)
    ks = d.sub(2).below(k_hi + 1, 0, count)
    dens = d.sub(3).uniform(0, count) * dens_hi
    pats = [random_pattern(d.sub(1000 + i), int(ms[i]), int(round(dens[i] * ms[i])))
            for i in range(count)]
    return pats, [int(x) for x in ks]


def plant_pool(text: np.ndarray, pats, ks, seed: int = SEED0 + 4):
    """Plant each query once (d ~ U{0..k}) in its own segment of the text."""
    d = Draws(key(seed, STREAM_PLANTS))
    slots = plant_slots(text.size, max(len(p) for p in pats), len(pats), d.sub(0))
    dd = d.sub(1).u64(0, len(pats))
    plants = []
    for i, pos in enumerate(slots):
        dist = int(dd[i] % np.uint64(ks[i] + 1))
        dist = plant(text, pos, pats[i], dist, d.sub(100 + i))
        plants.append((i, pos, dist))
    return plants


def poisson_arrivals(rate: float, duration: float, seed: int = SEED0 + 4) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate on [0, duration)."""
    d = Draws(key(seed, STREAM_ARRIVALS)).sub(int(rate * 1000))
    est = int(rate * duration * 1.5 + 100)
    u = d.uniform(0, est)
    t = np.cumsum(-np.log1p(-u) / rate)
    while t[-1] < duration:
        est *= 2
        u = d.uniform(0, est)
        t = np.cumsum(-np.log1p(-u) / rate)
    return t[t < duration]


def served(n: int = 3_100_000_000, count: int = 20000, text: np.ndarray | None = None) -> Workload:
    """The genome-scale text with the query pool planted in it (one copy per
    query, d ~ U{0..k}, in its own text segment), before it is made resident."""
    g = genome(n, text=text)
    pats, ks = query_pool(count)
    plants = plant_pool(g.text, pats, ks)
    return Workload("served", g.seed, n, g.text, pats, ks, plants)
