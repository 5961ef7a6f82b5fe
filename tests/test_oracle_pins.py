"""Pins for the oracle: values the paper prints, closed forms, brute force.

Each test ties the oracle (the C brute force in oracle/oracle.c and the
pure-Python routes in oracle/reference.py) to something other than itself.
"""
import itertools
import random

import numpy as np
import pytest

import oracle
from oracle import reference as ref
from conftest import golden_dict, golden_lines

SYMBOLS = "ACGTMRWSYKVHDBN-"


def c_counts(text, pattern):
    return oracle.counts(text, oracle.parse(pattern)).tolist()


def c_hits(text, pattern, k, threads=1):
    pos, cnt, total = oracle.scan(text, oracle.parse(pattern), k, threads=threads)
    assert total == len(pos)
    return list(zip(pos.tolist(), cnt.tolist()))


# --- worked examples --------------------------------------------------------

@pytest.mark.parametrize("fixture", ["example_sect1_1.txt", "example_sect2_5.txt"])
def test_worked_example_locations(fixture):
    """Sect. 1.1 and Sect. 2.5: exact match at location 5; with k = 2 also 1, 4, 6."""
    g = golden_dict(fixture)
    text, pattern = g["text"][0][0], g["pattern"][0][0]
    want0 = [int(x) - 1 for x in g["locations_k0"][0]]
    want2 = [int(x) - 1 for x in g["locations_k2"][0]]
    for k, want in ((0, want0), (2, want2)):
        assert [p for p, _ in c_hits(text, pattern, k)] == want
        assert [p for p, _ in ref.scan(text, ref.parse(pattern), k)] == want
    # k = 1 adds nothing: every approximate hit of the examples has 2 mismatches
    assert [p for p, _ in c_hits(text, pattern, 1)] == want0


def test_table4_pair_values_and_early_stop():
    """Table 4: each printed pair value equals the oracle's mismatch indicator,
    and each window lists exactly the pairs evaluated before the count passed k."""
    g = golden_dict("example_sect2_5.txt")
    text, pattern, k = g["text"][0][0], g["pattern"][0][0], int(g["k"][0][0])
    sets = ref.parse(pattern)
    for row in g["table4"]:
        loc = int(row[0])
        vi = row.index("value")
        values = [int(x) for x in row[vi + 1:]]
        mine = [0 if text[loc - 1 + j] in sets[j] else 1 for j in range(len(sets))]
        assert values == mine[:len(values)]
        # stop rule: evaluation ends at the first prefix whose count exceeds k
        c, stop = 0, len(sets)
        for j, v in enumerate(mine):
            c += v
            if c > k:
                stop = j + 1
                break
        assert len(values) == stop


def test_worked_example_full_counts():
    """Full counts of the Sect. 2.5 windows agree with Table 4 where it is
    complete (windows 1, 4, 5, 6) and exceed k where it stops early."""
    g = golden_dict("example_sect2_5.txt")
    text, pattern = g["text"][0][0], g["pattern"][0][0]
    full = c_counts(text, pattern)
    assert full == ref.full_counts(text, ref.parse(pattern))
    for row in g["table4"]:
        loc = int(row[0])
        vals = [int(x) for x in row[row.index("value") + 1:]]
        if len(vals) == len(pattern.replace("[CGT]", "B").replace("[CG]", "S")):
            assert full[loc - 1] == sum(vals)
        else:
            assert full[loc - 1] > 2


# --- Table 3 as prime divisibility -----------------------------------------

def test_table3_is_membership_and_prime_divisibility():
    """Every printed Table 3 value equals [t not in class] from the IUPAC
    meanings, and equals [q_t does not divide the class prime product] with
    q = (2, 3, 5, 7) and the empty class '-' given product 1."""
    rows = golden_lines("table3_pair_values.txt")
    assert len(rows) == 16
    for row in rows:
        sym, vals = row[0], [int(x) for x in row[1:5]]
        members = ref.IUPAC[sym]
        for b, v in zip("ACGT", vals):
            assert v == (0 if b in members else 1)
            assert v == ref.prime_pair_value(members, b)
        # and the C oracle's class for the same letter gives the same row
        s = int(oracle.parse(sym)[0])
        assert [0 if (s >> i) & 1 else 1 for i in range(4)] == vals


def test_prime_route_counts_match_bruteforce():
    rnd = random.Random(7)
    for _ in range(200):
        m = rnd.randint(1, 6)
        pat = "".join(rnd.choice(SYMBOLS) for _ in range(m))
        text = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(m, 30)))
        sets = ref.parse(pat)
        assert ref.prime_counts(text, sets) == c_counts(text, pat) == ref.full_counts(text, sets)


# --- Linhart-Shamir route (Sect. 1.3) ---------------------------------------

def test_crt_route_matches_bruteforce():
    """Eqs. (1)-(3) with big integers: exact hits are C_i mod M = 0, and the
    per-prime residues decode to the exact mismatch counts."""
    rnd = random.Random(11)
    for _ in range(150):
        m = rnd.randint(1, 6)
        pat = "".join(rnd.choice(SYMBOLS) for _ in range(m))
        text = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(m, 24)))
        sets = ref.parse(pat)
        primes = dict(zip("ACGT", ref.primes_above(m)))
        full = c_counts(text, pat)
        assert ref.crt_counts(text, sets, primes) == full
        assert ref.crt_exact_positions(text, sets, primes) == [i for i, c in enumerate(full) if c == 0]


def test_crt_class_codes_satisfy_eq1():
    primes = dict(zip("ACGT", ref.primes_above(5)))
    big_m = 1
    for v in primes.values():
        big_m *= v
    for sym, members in ref.IUPAC.items():
        n_s = ref.crt_class_code(members, primes)
        assert 0 <= n_s < big_m
        for b, kb in primes.items():
            assert n_s % kb == (0 if b in members else 1)


def test_sect2_5_example_through_crt_route():
    g = golden_dict("example_sect2_5.txt")
    text, pattern = g["text"][0][0], g["pattern"][0][0]
    sets = ref.parse(pattern)
    primes = dict(zip("ACGT", ref.primes_above(len(sets))))
    assert ref.crt_exact_positions(text, sets, primes) == [int(g["locations_k0"][0][0]) - 1]


def test_ls_precision_limit_sect1_3_5():
    """m = 1000: primes 1009..1021, M ~ 1e12, text codes ~ 1e9, and a class
    code times a text code can exceed uint64."""
    g = golden_dict("ls_precision_sect1_3_5.txt")
    m = int(g["m"][0][0])
    want = [int(x) for x in g["primes"][0]]
    assert ref.primes_above(m) == want
    primes = dict(zip("ACGT", want))
    big_m = want[0] * want[1] * want[2] * want[3]
    assert 1e12 <= big_m < 2e12
    assert all(0.9e9 < big_m // q < 1.1e9 for q in want)
    worst = max(ref.crt_class_code(s, primes) for s in ref.IUPAC.values()) * max(big_m // q for q in want)
    assert worst > 2 ** 64 - 1


# --- closed forms and brute force -------------------------------------------

def test_de_bruijn_holds_every_mer_once():
    for order in range(1, 7):
        s = ref.de_bruijn(order)
        assert len(s) == 4 ** order + order - 1
        mers = {s[i:i + order] for i in range(4 ** order)}
        assert len(mers) == 4 ** order


def test_debruijn_histogram_closed_form():
    """On a text holding every m-mer once, the count histogram is the
    coefficient list of prod_j (|S_j| + (4 - |S_j|) x)."""
    rnd = random.Random(3)
    for m in range(1, 8):
        text = ref.de_bruijn(m)
        for _ in range(6):
            pat = "".join(rnd.choice(SYMBOLS) for _ in range(m))
            full = c_counts(text, pat)
            hist = np.bincount(full, minlength=m + 1).tolist()
            assert hist == ref.debruijn_histogram(ref.parse(pat))


@pytest.mark.parametrize("m", [1, 2, 3])
def test_exhaustive_small_patterns(m):
    """Every pattern of length m over the 16 symbols, against every m-mer (a
    de Bruijn text), for every k: the early-stopping C oracle equals the
    pure-Python full count filtered by k."""
    text = ref.de_bruijn(m)
    for tup in itertools.product(SYMBOLS, repeat=m):
        pat = "".join(tup)
        full = ref.full_counts(text, ref.parse(pat))
        for k in range(m + 1):
            want = [(i, c) for i, c in enumerate(full) if c <= k]
            assert c_hits(text, pat, k) == want


def test_all_short_texts():
    """All 4^6 texts of length 6 against a fixed set of patterns, every k."""
    pats = ["ACG", "N-T", "[AC]GY", "BDHV", "-", "NNNN"]
    for tup in itertools.product("ACGT", repeat=6):
        text = "".join(tup)
        for pat in pats:
            sets = ref.parse(pat)
            full = ref.full_counts(text, sets)
            assert c_counts(text, pat) == full


# --- textbook special cases -------------------------------------------------

def test_exact_singletons_equal_string_search():
    rnd = random.Random(5)
    for _ in range(100):
        text = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(20, 400)))
        m = rnd.randint(1, 6)
        pat = "".join(rnd.choice("ACGT") for _ in range(m))
        want, i = [], text.find(pat)
        while i >= 0:
            want.append(i)
            i = text.find(pat, i + 1)
        assert [p for p, _ in c_hits(text, pat, 0)] == want


def test_all_n_all_dash_and_large_k():
    text = "ACGTTGCAACGGTACCA"
    n = len(text)
    assert c_counts(text, "NNNN") == [0] * (n - 3)
    assert c_counts(text, "----") == [4] * (n - 3)
    assert c_hits(text, "----", 3) == []
    hits = c_hits(text, "GATTACA", 7)
    assert len(hits) == n - 7 + 1 and [p for p, _ in hits] == list(range(n - 6))


# --- invariants -------------------------------------------------------------

def test_invariants():
    rnd = random.Random(9)
    for _ in range(60):
        m = rnd.randint(1, 12)
        pat = "".join(rnd.choice(SYMBOLS) for _ in range(m))
        text = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(m, 200)))
        sets = ref.parse(pat)
        full = c_counts(text, pat)
        # monotone in k
        prev = set()
        for k in range(m + 1):
            cur = {p for p, _ in c_hits(text, pat, k)}
            assert prev <= cur
            prev = cur
        # additivity over a split of the pattern
        if m >= 2:
            cut = rnd.randint(1, m - 1)
            a = ref.full_counts(text[:len(text) - (m - cut)], sets[:cut])
            b = ref.full_counts(text[cut:], sets[cut:])
            assert full == [x + y for x, y in zip(a, b)]
        # reverse complement: window i maps to window n-m-i
        rc = ref.full_counts(ref.reverse_complement_text(text), ref.reverse_complement_sets(sets))
        assert rc == full[::-1]
        # relabelling the bases consistently in text and classes
        perm = dict(zip("ACGT", rnd.sample("ACGT", 4)))
        t2 = "".join(perm[c] for c in text)
        s2 = [frozenset(perm[b] for b in s) for s in sets]
        assert ref.full_counts(t2, s2) == full


def test_thread_partition_and_ranges():
    """Sect. 2.6: splitting the windows over threads (each range reading m-1
    extra bases) gives the same list; window sub-ranges are slices of it."""
    rnd = random.Random(13)
    text = "".join(rnd.choice("ACGT") for _ in range(5000))
    pat = "AC[GT]NNA-CG"
    sets = oracle.parse(pat)
    base = oracle.scan(text, sets, 5, threads=1)
    for t in (2, 3, 5, 8, 64):
        got = oracle.scan(text, sets, 5, threads=t)
        assert got[2] == base[2]
        assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])
    for b, e in ((0, 10), (17, 4000), (4990, 10 ** 9), (100, 100)):
        pos, cnt, total = oracle.scan(text, sets, 5, threads=3, win_begin=b, win_end=e)
        sel = (base[0] >= b) & (base[0] < e)
        assert np.array_equal(pos, base[0][sel]) and np.array_equal(cnt, base[1][sel])


def test_capacity_protocol():
    text = "ACGT" * 50
    pos, cnt, total = oracle.scan(text, oracle.parse("NN"), 0, capacity=7)
    assert total == 199 and pos.tolist() == list(range(7)) and cnt.tolist() == [0] * 7


def test_error_conventions():
    with pytest.raises(oracle.OracleError):
        oracle.scan("ACGTX", oracle.parse("AC"), 0)
    with pytest.raises(oracle.OracleError):
        oracle.parse("A[]C")
    with pytest.raises(oracle.OracleError):
        oracle.parse("AZ")
    with pytest.raises(oracle.OracleError):
        oracle.scan("ACGT", oracle.parse("AC"), 70000)
    assert oracle.first_bad(b"ACGTacgtN") == 8
    assert oracle.scan("ACG", oracle.parse("ACGT"), 4)[2] == 0        # m > n
    assert oracle.scan("ACGT", oracle.parse("ACGA"), 1)[2] == 1       # m == n
    assert list(oracle.parse("ac[gt]n-")) == list(oracle.parse("AC[TG]N-"))


def test_bracket_classes_canonical():
    """A bracket class is the union of its letters: [CGT] is B, [CG] is S."""
    assert list(oracle.parse("[CGT][CG][AC][ACGT]")) == list(oracle.parse("BSMN"))
    assert ref.parse("[CGT][CG]") == ref.parse("BS")


def test_planted_sites_have_their_distance():
    from paper_1611_06115_amd import synth

    w = synth.small()
    sets = oracle.parse(w.patterns[0])
    for _, pos, d in w.plants:
        assert oracle.counts(w.text[pos:pos + sets.size], sets).tolist() == [d]
    pos, cnt, _ = oracle.scan(w.text, sets, 2, threads=4)
    found = dict(zip(pos.tolist(), cnt.tolist()))
    for _, p, d in w.plants:
        if d <= 2:
            assert found[p] == d


# --- planted mistakes: the pins above must catch a broken oracle -------------

def _mutants():
    def off_by_one(text, sets):
        t = ref._text(text)
        m = len(sets)
        return [sum(1 for j in range(m) if t[min(i + j + 1, len(t) - 1)] not in sets[j])
                for i in range(len(t) - m + 1)]

    def dropped_last(text, sets):
        t = ref._text(text)
        m = len(sets)
        return [sum(1 for j in range(m - 1) if t[i + j] not in sets[j]) for i in range(len(t) - m + 1)]

    def reversed_pattern(text, sets):
        return ref.full_counts(text, list(reversed(sets)))

    def complement_class(text, sets):
        return ref.full_counts(text, [frozenset("ACGT") - s for s in sets])

    def dash_matches(text, sets):
        return ref.full_counts(text, [s or frozenset("ACGT") for s in sets])

    return [off_by_one, dropped_last, reversed_pattern, complement_class, dash_matches]


@pytest.mark.parametrize("mutant", _mutants(), ids=lambda f: f.__name__)
def test_pins_catch_planted_mistakes(mutant):
    caught = False
    for fx in ("example_sect1_1.txt", "example_sect2_5.txt"):
        g = golden_dict(fx)
        text, pattern = g["text"][0][0], g["pattern"][0][0]
        got = [i for i, c in enumerate(mutant(text, ref.parse(pattern))) if c <= 2]
        caught |= got != [int(x) - 1 for x in g["locations_k2"][0]]
    for m in (3, 4):
        text = ref.de_bruijn(m)
        for pat in ("AC-", "B-NT", "GGT", "[AC]T-G"):
            if len(ref.parse(pat)) != m:
                continue
            hist = np.bincount(mutant(text, ref.parse(pat)), minlength=m + 1).tolist()
            caught |= hist != ref.debruijn_histogram(ref.parse(pat))
    assert caught


def test_fasta_reading_pinned_by_hand():
    """The FASTA reading (records separate, lower case folded, a window
    covering a non-ACGT letter or crossing records has no count): the
    oracle's two routes give the hits worked out by hand in
    tests/golden/fasta_reading.txt."""
    from oracle import reference as ref

    rows = golden_lines("fasta_reading.txt")
    fa = "\n".join(" ".join(r[1:]) for r in rows if r[0] == "fasta") + "\n"
    for r in rows:
        if r[0] != "query":
            continue
        p, k = r[1], int(r[2])
        want = [] if r[3:] == ["none"] else [tuple(map(int, x.split(":"))) for x in r[3:]]
        assert ref.fasta_scan(fa, ref.parse(p), k) == want, p
        pos, cnt = oracle.fasta_scan(fa.encode(), p, k)
        assert list(zip(pos.tolist(), cnt.tolist())) == want, p


def test_fasta_reading_reduces_to_the_plain_scan():
    """One record of A/C/G/T only is the plain scan of its sequence; upper
    and lower case give the same hits; splitting a record at an unknown
    letter gives the hits of the two parts (offsets shifted)."""
    import random

    from oracle import reference as ref

    rnd = random.Random(11)
    seq = "".join(rnd.choice("ACGT") for _ in range(400))
    sets = ref.parse("A[CG]TN-G"[:5] + "AC")
    for k in range(4):
        plain = ref.scan(seq, sets, k)
        assert ref.fasta_scan(">x\n" + seq + "\n", sets, k) == plain
        assert ref.fasta_scan(">x\n" + seq.lower() + "\n", sets, k) == plain
        cut = 173
        split = ref.fasta_scan(">x\n" + seq[:cut] + "N" + seq[cut + 1:] + "\n", sets, k)
        left = ref.scan(seq[:cut], sets, k)
        right = [(i + cut + 1, c) for i, c in ref.scan(seq[cut + 1:], sets, k)]
        assert split == left + right
