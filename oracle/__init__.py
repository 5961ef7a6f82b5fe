"""Oracle for the k-mismatch character-class scan -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package.  The product path (``paper_1611_06115_amd``)
never imports it, and it imports nothing from the product path: the two
share no code, header, table or helper.

Two implementations live here, both written from the paper's definitions:

* ``oracle.c`` (built to ``liboracle.so`` with gcc): the multithreaded brute
  force with the early stop of Sect. 2.4 and the range partition of Sect. 2.6.
  ``scan`` below calls it.
* ``reference.py``: pure-Python routes for small inputs (full counts without
  early stop, prime divisibility, the Linhart-Shamir CRT route of Sect. 1.3,
  and the de Bruijn closed form).

Pins (see tests/test_oracle_*.py) tie both to values the paper prints and to
closed forms, so neither is trusted on its own word.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import reference  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain C, gcc, -O2, pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64, i64, p = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        lib.pmo_parse.argtypes = [ctypes.c_char_p, u64, p, u64]
        lib.pmo_parse.restype = i64
        lib.pmo_first_bad.argtypes = [p, u64]
        lib.pmo_first_bad.restype = i64
        lib.pmo_counts.argtypes = [p, u64, p, u64, p]
        lib.pmo_counts.restype = ctypes.c_int
        lib.pmo_scan_range.argtypes = [p, u64, p, u64, u64, u64, u64, ctypes.c_int, p, p, u64]
        lib.pmo_scan_range.restype = i64
        _lib = lib
    return _lib


class OracleError(ValueError):
    pass


def _as_u8(text) -> np.ndarray:
    if isinstance(text, str):
        text = text.encode("ascii")
    if isinstance(text, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(text), dtype=np.uint8)
    arr = np.ascontiguousarray(np.asarray(text), dtype=np.uint8)
    return arr


def parse(pattern: str) -> np.ndarray:
    """Pattern -> uint8 member sets (bit b set <=> base b of A,C,G,T matches)."""
    raw = pattern.encode("ascii")
    lib = _load()
    m = lib.pmo_parse(raw, len(raw), None, 0)
    if m < 0:
        raise OracleError(f"bad pattern {pattern!r}")
    sets = np.zeros(max(m, 1), dtype=np.uint8)
    lib.pmo_parse(raw, len(raw), sets.ctypes.data, m)
    return sets[:m]


def first_bad(text) -> int:
    t = _as_u8(text)
    return int(_load().pmo_first_bad(t.ctypes.data, t.size))


def counts(text, sets) -> np.ndarray:
    """Full counts of every window (no early stop); small inputs only."""
    t = _as_u8(text)
    s = np.ascontiguousarray(sets, dtype=np.uint8)
    nw = max(t.size - s.size + 1, 0)
    out = np.zeros(max(nw, 1), dtype=np.uint32)
    rc = _load().pmo_counts(t.ctypes.data, t.size, s.ctypes.data, s.size, out.ctypes.data)
    if rc != 0:
        raise OracleError(f"oracle counts failed ({rc})")
    return out[:nw]


def scan(text, sets, k: int, threads: int = 1, win_begin: int = 0, win_end: int | None = None,
         capacity: int | None = None):
    """Brute-force scan.  Returns (positions int64, counts uint16, total hits).

    ``sets`` is the output of ``parse`` (or any uint8 member-set array)."""
    t = _as_u8(text)
    s = np.ascontiguousarray(sets, dtype=np.uint8)
    lib = _load()
    end = np.iinfo(np.uint64).max if win_end is None else int(win_end)
    if capacity is None:
        total = lib.pmo_scan_range(t.ctypes.data, t.size, s.ctypes.data, s.size, int(k),
                                   int(win_begin), end, int(threads), None, None, 0)
        if total < 0:
            raise OracleError(f"oracle scan failed ({total})")
        capacity = int(total)
    pos = np.zeros(max(capacity, 1), dtype=np.int64)
    cnt = np.zeros(max(capacity, 1), dtype=np.uint16)
    total = lib.pmo_scan_range(t.ctypes.data, t.size, s.ctypes.data, s.size, int(k),
                               int(win_begin), end, int(threads), pos.ctypes.data,
                               cnt.ctypes.data, capacity)
    if total < 0:
        raise OracleError(f"oracle scan failed ({total})")
    kept = min(int(total), capacity)
    return pos[:kept], cnt[:kept], int(total)


def fasta_scan(data: bytes, pattern: str, k: int, threads: int = 1):
    """The FASTA reading (see reference.fasta_scan) for larger inputs: records
    split into maximal runs of A/C/G/T, each run scanned by the brute force
    above, positions shifted to offsets in the records' concatenation.
    Returns (positions int64, counts uint16)."""
    sets = parse(pattern)
    m = len(sets)
    text = data.decode("ascii") if isinstance(data, (bytes, bytearray)) else data
    pos_all, cnt_all = [], []
    offset = 0
    for _, seq in reference.fasta_records(text):
        i = 0
        while i < len(seq):
            if seq[i] not in "ACGT":
                i += 1
                continue
            j = i
            while j < len(seq) and seq[j] in "ACGT":
                j += 1
            if j - i >= m:
                pos, cnt, _ = scan(seq[i:j], sets, k, threads=threads)
                pos_all.append(pos + offset + i)
                cnt_all.append(cnt)
            i = j
        offset += len(seq)
    if not pos_all:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.uint16)
    return np.concatenate(pos_all), np.concatenate(cnt_all)


def hardware_threads() -> int:
    return os.cpu_count() or 1
