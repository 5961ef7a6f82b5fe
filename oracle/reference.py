"""Pure-Python routes of the oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's cpu_baseline leg use this
module.  Each function is an independent, deliberately plain route to the
quantities the scan defines, for small inputs:

* ``parse`` -- pattern string -> list of member-base sets, from the IUPAC
  meanings of Table 2 (first column) and the bracket notation of the examples
  in Sect. 1.1 and 2.5.
* ``full_counts`` -- c_i = #{j : t[i+j] not in S_j} for every window, with no
  early stop (the class-match and k-mismatch definitions of Sect. 1.1).
* ``scan`` -- [(i, c_i)] with c_i <= k, ascending i.
* ``prime_pair_value`` / ``prime_counts`` -- the same counts reached through
  prime coding: base b gets prime q_b, a class the product of its members'
  primes, and a pair mismatches when q_t does not divide the class product.
  This is the pair dictionary of Table 3 (Sect. 2.3), read as divisibility.
* ``crt_counts`` -- the Linhart-Shamir route of Sect. 1.3 (eqs. 1-3): CRT
  codes n_S for classes, e_b = M/k_b for bases, the correlation C_i, and
  exact matches where C_i mod M = 0.  Counts are decoded per prime.
* ``de_bruijn`` / ``debruijn_histogram`` -- a text holding every L-mer once and
  the closed-form count histogram prod_j (|S_j| + (4-|S_j|) x).

Positions are 0-based here; the paper's location i is position i-1.
"""
from __future__ import annotations

from math import prod

BASES = "ACGT"

# IUPAC one-letter classes (Table 2, first column); '-' matches nothing.
IUPAC = {
    "A": "A", "C": "C", "G": "G", "T": "T",
    "M": "AC", "R": "AG", "W": "AT", "S": "CG", "Y": "CT", "K": "GT",
    "V": "ACG", "H": "ACT", "D": "AGT", "B": "CGT",
    "N": "ACGT", "-": "",
}


def parse(pattern: str) -> list[frozenset]:
    """Pattern string -> list of member sets (upper-case base letters)."""
    out: list[frozenset] = []
    i = 0
    while i < len(pattern):
        ch = pattern[i]
        if ch == "[":
            j = pattern.index("]", i + 1)
            inner = pattern[i + 1:j]
            if not inner:
                raise ValueError("empty class []")
            members: set = set()
            for c in inner:
                c = c.upper()
                if c == "-" or c not in IUPAC:
                    raise ValueError(f"bad class member {c!r}")
                members |= set(IUPAC[c])
            out.append(frozenset(members))
            i = j + 1
        else:
            c = ch.upper()
            if c not in IUPAC:
                raise ValueError(f"bad pattern symbol {ch!r}")
            out.append(frozenset(IUPAC[c]))
            i += 1
    return out


def _text(text) -> str:
    if isinstance(text, (bytes, bytearray, memoryview)):
        text = bytes(text).decode("ascii")
    t = text.upper()
    bad = [i for i, c in enumerate(t) if c not in BASES]
    if bad:
        raise ValueError(f"bad text symbol at {bad[0]}")
    return t


def full_counts(text, sets: list) -> list[int]:
    """Mismatch count of every window, no early stop."""
    t = _text(text)
    m = len(sets)
    if m == 0:
        raise ValueError("empty pattern")
    return [sum(1 for j in range(m) if t[i + j] not in sets[j])
            for i in range(len(t) - m + 1)]


def scan(text, sets: list, k: int) -> list[tuple[int, int]]:
    """All (position, count) with count <= k, ascending."""
    return [(i, c) for i, c in enumerate(full_counts(text, sets)) if c <= k]


# --- prime coding (Table 3 read as divisibility) ---------------------------

SMALL_PRIMES = {"A": 2, "C": 3, "G": 5, "T": 7}


def class_product(members, primes=SMALL_PRIMES) -> int:
    """Product of the primes of a class's members; the empty class gives 1."""
    return prod(primes[b] for b in members)


def prime_pair_value(members, base: str, primes=SMALL_PRIMES) -> int:
    """0 when the base's prime divides the class product (a match), else 1."""
    return 0 if class_product(members, primes) % primes[base] == 0 else 1


def prime_counts(text, sets: list, primes=SMALL_PRIMES) -> list[int]:
    t = _text(text)
    m = len(sets)
    prods = [class_product(s, primes) for s in sets]
    return [sum(0 if prods[j] % primes[t[i + j]] == 0 else 1 for j in range(m))
            for i in range(len(t) - m + 1)]


# --- Linhart-Shamir CRT route (Sect. 1.3, eqs. 1-3) ------------------------

def crt_class_code(members, primes: dict) -> int:
    """n_S with n_S = 0 mod k_b for b in S and n_S = 1 mod k_b otherwise (eq. 1),
    the unique such integer in [0, M)."""
    big_m = prod(primes.values())
    n_s = 0
    for b, kb in primes.items():
        r = 0 if b in members else 1
        mb = big_m // kb
        n_s += r * mb * pow(mb, -1, kb)
    return n_s % big_m


def crt_correlation(text, sets: list, primes: dict) -> list[int]:
    """C_i = sum_j n_{S_j} * e_{t[i+j]}, e_b = M / k_b.

    Eq. (2) is printed as a convolution; matching window i against the pattern
    needs the pattern read forwards, i.e. a correlation, which is used here."""
    t = _text(text)
    big_m = prod(primes.values())
    codes = [crt_class_code(s, primes) for s in sets]
    e = {b: big_m // kb for b, kb in primes.items()}
    m = len(sets)
    return [sum(codes[j] * e[t[i + j]] for j in range(m)) for i in range(len(t) - m + 1)]


def crt_exact_positions(text, sets: list, primes: dict) -> list[int]:
    """Eq. (3): exact occurrences are the windows with C_i mod M = 0."""
    big_m = prod(primes.values())
    return [i for i, c in enumerate(crt_correlation(text, sets, primes)) if c % big_m == 0]


def crt_counts(text, sets: list, primes: dict) -> list[int]:
    """Mismatch counts decoded from C_i: modulo k_b only the terms whose text
    base is b survive, each contributing (M/k_b) * [b not in S_j]; as the count
    is below k_b (all primes exceed m) it is (C_i mod k_b) * (M/k_b)^-1 mod k_b."""
    big_m = prod(primes.values())
    out = []
    for c in crt_correlation(text, sets, primes):
        total = 0
        for kb in primes.values():
            mb = big_m // kb
            total += (c % kb) * pow(mb, -1, kb) % kb
        out.append(total)
    return out


def primes_above(m: int, count: int = 4) -> list[int]:
    """The `count` smallest primes larger than m (Sect. 1.3 needs all > m)."""
    out = []
    x = m + 1
    while len(out) < count:
        if x >= 2 and all(x % d for d in range(2, int(x ** 0.5) + 1)):
            out.append(x)
        x += 1
    return out


# --- de Bruijn closed form --------------------------------------------------

def de_bruijn(order: int, alphabet: str = BASES) -> str:
    """Linear de Bruijn sequence: every string of length `order` over the
    alphabet occurs exactly once as a substring (cyclic sequence built from
    the concatenation of Lyndon words in lexicographic order, then its first
    order-1 symbols appended)."""
    kk = len(alphabet)
    a = [0] * (kk * order)
    seq: list[int] = []

    def db(t: int, p: int) -> None:
        if t > order:
            if order % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, kk):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    cyc = "".join(alphabet[i] for i in seq)
    return cyc + cyc[:order - 1]


def debruijn_histogram(sets: list) -> list[int]:
    """Coefficients of prod_j (|S_j| + (4 - |S_j|) x): over all 4^m window
    contents, how many have exactly c mismatches."""
    poly = [1]
    for s in sets:
        a, b = len(s), 4 - len(s)
        nxt = [0] * (len(poly) + 1)
        for i, v in enumerate(poly):
            nxt[i] += v * a
            nxt[i + 1] += v * b
        poly = nxt
    return poly


def reverse_complement_text(text: str) -> str:
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    return "".join(comp[c] for c in reversed(_text(text)))


def reverse_complement_sets(sets: list) -> list[frozenset]:
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    return [frozenset(comp[b] for b in s) for s in reversed(sets)]


# --- FASTA input -------------------------------------------------------------
#
# Reading (the paper is silent; Sect. 3 scans a chromosome FASTA file and
# Table 1 codes only A, C, G, T): records are separate texts; lower case is
# the same base; any other sequence letter is an unknown base, for which
# eq. (4) has no pair value, so a window covering one has no count; a window
# never spans two records.  Positions are offsets in the concatenation of
# the records' letters (line breaks and headers removed).

def fasta_records(data: str) -> list[tuple[str, str]]:
    """(name, sequence) per '>' record; sequence letters upper-cased, line
    breaks and blanks dropped; ';' lines are comments."""
    records: list[tuple[str, list[str]]] = []
    for line in data.splitlines():
        if line.startswith(">"):
            fields = line[1:].split()
            records.append((fields[0] if fields else "", []))
        elif line.startswith(";"):
            continue
        else:
            letters = "".join(line.split())
            if letters:
                if not records:
                    raise ValueError("sequence before the first header")
                records[-1][1].append(letters.upper())
    return [(name, "".join(parts)) for name, parts in records]


def fasta_scan(data: str, sets: list, k: int) -> list[tuple[int, int]]:
    """[(offset, c)] for every window inside one record, made only of the
    bases A, C, G, T, with c = #{j : t[i+j] not in S_j} <= k; ascending."""
    m = len(sets)
    out = []
    offset = 0
    for _, seq in fasta_records(data):
        for i in range(len(seq) - m + 1):
            window = seq[i:i + m]
            if all(ch in BASES for ch in window):
                c = sum(1 for j in range(m) if window[j] not in sets[j])
                if c <= k:
                    out.append((offset + i, c))
        offset += len(seq)
    return out
