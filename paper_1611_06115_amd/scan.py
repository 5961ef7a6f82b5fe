"""ctypes binding of libpmscan (include/pmscan.h): argument marshalling only.

Every step of the scan runs in the HIP library; torch provides device memory
(tensors) and streams.  Loading fails loudly when the library is missing:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmscan.so")
_lib = None
UINT64_MAX = (1 << 64) - 1


class PMError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_name(status)}: {detail}")
        self.status = status
        self.detail = detail


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        u8p, u16p, u32p, u64p = (ctypes.POINTER(t) for t in
                                 (ctypes.c_uint8, ctypes.c_uint16, ctypes.c_uint32, ctypes.c_uint64))
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        sig = {
            "pm_status_string": ([i32], ctypes.c_char_p),
            "pm_last_error_detail": ([], ctypes.c_char_p),
            "pm_version": ([], ctypes.c_char_p),
            "pm_text_bytes": ([u64], u64),
            "pm_encode_text": ([vp, u64, vp, vp, vp], i32),
            "pm_encode_pattern": ([ctypes.c_char_p, u64, vp, u64, u32p], i32),
            "pm_pair_table": ([vp], i32),
            "pm_pattern_bytes": ([u32], u64),
            "pm_pattern_image": ([vp, u32, vp, u64], i32),
            "pm_scan_workspace_bytes": ([u64], u64),
            "pm_scan": ([vp, u64, vp, u32, u32, vp, u64, u64, vp, vp, u64, vp, vp, u64, vp], i32),
            "pm_scan_noalloc_max_windows": ([], u64),
            "pm_scan_noalloc": ([vp, u64, vp, u32, u32, vp, u64, u64, vp, vp, u64, vp, vp], i32),
            "pm_expected_hits": ([vp, u32, u32, u64, ctypes.POINTER(ctypes.c_double)], i32),
            "pm_fasta_parse": ([ctypes.c_char_p, u64, ctypes.POINTER(vp)], i32),
            "pm_fasta_free": ([vp], None),
            "pm_fasta_length": ([vp], u64),
            "pm_fasta_bases": ([vp], vp),
            "pm_fasta_record_count": ([vp], u32),
            "pm_fasta_record": ([vp, u32, ctypes.POINTER(ctypes.c_char_p), u64p, u64p], i32),
            "pm_fasta_unknown_run_count": ([vp], u64),
            "pm_fasta_unknown_run": ([vp, u64, u64p, u64p], i32),
            "pm_fasta_window_ranges": ([vp, u32, vp, vp, u64, u64p], i32),
            "pm_scan_fasta_workspace_bytes": ([vp], u64),
            "pm_scan_fasta": ([vp, vp, vp, u32, u32, vp, vp, vp, u64, u64p, vp, u64, vp], i32),
            "pm_scan_batch_workspace_bytes": ([u64, u32, vp, vp, vp], u64),
            "pm_scan_batch": ([vp, u64, u32, vp, vp, vp, vp, vp, u64, u64, vp, vp, vp, vp, vp, u64, vp, vp],
                              i32),
            "pm_time_next_scan": ([vp, vp], i32),
            "pm_crt_counts_workspace_bytes": ([u64, u32], u64),
            "pm_crt_counts": ([vp, u64, vp, u32, vp, vp, u64, vp], i32),
            "pm_scan_host_workspace_bytes": ([u64, u32], u64),
            "pm_scan_host": ([vp, u64, vp, u32, u32, vp, u64, vp, vp, u64, vp, vp, u64, vp, vp], i32),
            "pm_server_now_ns": ([], u64),
            "pm_server_min_arena_bytes": ([u64, vp], u64),
            "pm_server_create": ([vp, u64, vp, u64, vp, vp, vp], i32),
            "pm_server_submit": ([vp, vp, u32, u32, u64, vp], i32),
            "pm_server_poll": ([vp, u64, vp], i32),
            "pm_server_wait": ([vp, u64, ctypes.c_int64, vp], i32),
            "pm_server_release": ([vp, u64], i32),
            "pm_server_drain": ([vp, ctypes.c_int64], i32),
            "pm_server_stats_get": ([vp, vp], i32),
            "pm_server_error_detail": ([vp], ctypes.c_char_p),
            "pm_server_destroy": ([vp], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_name(status: int) -> str:
    return lib().pm_status_string(status).decode()


def check(status: int) -> None:
    if status != 0:
        raise PMError(status, lib().pm_last_error_detail().decode())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def time_next_scan(ev_begin, ev_end) -> None:
    """Have the next scan call of this thread record two torch.cuda.Event
    objects around its main kernel (events must have been recorded once, so
    that they exist)."""
    check(lib().pm_time_next_scan(ctypes.c_void_p(ev_begin.cuda_event), ctypes.c_void_p(ev_end.cuda_event)))


# --- host-side encoding (Tables 2 and 3) -------------------------------------

def encode_pattern(pattern: str) -> np.ndarray:
    """Pattern string -> Table 2 codes (uint8, 0..15)."""
    raw = pattern.encode("ascii")
    m = ctypes.c_uint32(0)
    check(lib().pm_encode_pattern(raw, len(raw), None, 0, ctypes.byref(m)))
    codes = np.zeros(max(m.value, 1), dtype=np.uint8)
    check(lib().pm_encode_pattern(raw, len(raw), codes.ctypes.data, codes.size, ctypes.byref(m)))
    return codes[:m.value]


def pair_table() -> np.ndarray:
    """The 64-entry pair dictionary of Table 3, derived from prime coding."""
    t = np.zeros(64, dtype=np.uint8)
    check(lib().pm_pair_table(t.ctypes.data))
    return t


def pattern_image(codes: np.ndarray) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    nbytes = lib().pm_pattern_bytes(codes.size)
    img = np.zeros(nbytes // 4, dtype=np.uint32)
    check(lib().pm_pattern_image(codes.ctypes.data, codes.size, img.ctypes.data, nbytes))
    return img


def text_bytes(n: int) -> int:
    return int(lib().pm_text_bytes(n))


def workspace_bytes(n: int) -> int:
    return int(lib().pm_scan_workspace_bytes(n))


# --- device objects ------------------------------------------------------------

@dataclass
class Text:
    """An encoded text resident in device memory."""
    data: "object"       # torch.uint8 tensor, pm_text_bytes(n) bytes
    n: int
    bad: "object"        # torch.int64 tensor [1]: first bad index, or -1

    def check(self) -> None:
        v = int(self.bad.item())
        if v != -1:
            raise PMError(-2, f"text byte {v} is not A, C, G or T")


class Pattern:
    """A parsed pattern: host codes plus a device image per device."""

    def __init__(self, pattern: str | np.ndarray):
        if isinstance(pattern, str):
            self.source = pattern
            self.codes = encode_pattern(pattern)
        else:
            self.source = None
            self.codes = np.ascontiguousarray(pattern, dtype=np.uint8)
        if self.codes.size == 0:
            raise PMError(-1, "empty pattern")
        self._images = {}

    @property
    def m(self) -> int:
        return int(self.codes.size)

    def image(self, device):
        import torch

        key = str(device)
        if key not in self._images:
            self._images[key] = torch.from_numpy(pattern_image(self.codes)).to(device)
        return self._images[key]


def encode_text(ascii, device=None, stream=None) -> Text:
    """Encode ASCII bases (torch uint8 tensor or numpy array) into device memory."""
    import torch

    if not isinstance(ascii, torch.Tensor):
        ascii = torch.from_numpy(np.ascontiguousarray(ascii, dtype=np.uint8))
    dev = torch.device(device) if device is not None else (
        ascii.device if ascii.is_cuda else torch.device("cuda"))
    if not ascii.is_cuda:
        ascii = ascii.to(dev, non_blocking=False)
    ascii = ascii.contiguous()
    n = int(ascii.numel())
    data = torch.empty(text_bytes(n), dtype=torch.uint8, device=dev)
    bad = torch.empty(1, dtype=torch.int64, device=dev)
    check(lib().pm_encode_text(ctypes.c_void_p(ascii.data_ptr()), n, ctypes.c_void_p(data.data_ptr()),
                               ctypes.c_void_p(bad.data_ptr()), _stream(stream)))
    return Text(data, n, bad)


class Workspace:
    """Reusable scan workspace and output buffers for one device."""

    def __init__(self, device, n: int, capacity: int = 1 << 16):
        import torch

        self.device = torch.device(device)
        self.ws = torch.empty(workspace_bytes(n), dtype=torch.uint8, device=self.device)
        self.n_hits = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.resize(capacity)

    def resize(self, capacity: int) -> None:
        import torch

        self.capacity = int(capacity)
        self.pos = torch.empty(max(self.capacity, 1), dtype=torch.int64, device=self.device)
        self.cnt = torch.empty(max(self.capacity, 1), dtype=torch.uint16, device=self.device)


def scan_async(text: Text, pattern: Pattern, k: int, ws: Workspace, win_begin: int = 0,
               win_end: int | None = None, stream=None) -> None:
    """Enqueue one pm_scan into ws (outputs ws.pos/ws.cnt/ws.n_hits)."""
    if win_end is None:
        win_end = UINT64_MAX
    img = pattern.image(text.data.device)
    check(lib().pm_scan(
        ctypes.c_void_p(text.data.data_ptr()), text.n, pattern.codes.ctypes.data, pattern.m, int(k),
        ctypes.c_void_p(img.data_ptr()), int(win_begin), int(win_end),
        ctypes.c_void_p(ws.pos.data_ptr()), ctypes.c_void_p(ws.cnt.data_ptr()), ws.capacity,
        ctypes.c_void_p(ws.n_hits.data_ptr()), ctypes.c_void_p(ws.ws.data_ptr()), ws.ws.numel(),
        _stream(stream)))


def noalloc_max_windows() -> int:
    """Windows one pm_scan_noalloc call may cover (its static scratch)."""
    return int(lib().pm_scan_noalloc_max_windows())


def scan_noalloc_async(text: Text, pattern: Pattern, k: int, pos, cnt, n_hits, win_begin: int = 0,
                       win_end: int | None = None, stream=None) -> None:
    """Enqueue one pm_scan_noalloc (no workspace: the library's static
    scratch) into caller tensors pos (int64), cnt (uint16) and n_hits (one
    int64); the capacity is pos.numel()."""
    if win_end is None:
        win_end = UINT64_MAX
    img = pattern.image(text.data.device)
    check(lib().pm_scan_noalloc(
        ctypes.c_void_p(text.data.data_ptr()), text.n, pattern.codes.ctypes.data, pattern.m, int(k),
        ctypes.c_void_p(img.data_ptr()), int(win_begin), int(win_end),
        ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), int(pos.numel()),
        ctypes.c_void_p(n_hits.data_ptr()), _stream(stream)))


def crt_counts_workspace_bytes(n: int, m: int) -> int:
    return int(lib().pm_crt_counts_workspace_bytes(int(n), int(m)))


def crt_counts(text: Text, pattern: Pattern | str, stream=None):
    """Every window's mismatch count by the transform route (pm_crt_counts):
    an int32 device tensor of n-m+1 counts (empty when m > n)."""
    import torch

    pattern = pattern if isinstance(pattern, Pattern) else Pattern(pattern)
    dev = text.data.device
    nw = text.n - pattern.m + 1 if pattern.m <= text.n else 0
    out = torch.empty(max(nw, 0), dtype=torch.int32, device=dev)
    ws = torch.empty(max(crt_counts_workspace_bytes(text.n, pattern.m), 256), dtype=torch.uint8, device=dev)
    crt_counts_into(text, pattern, out, ws, stream)
    return out


def crt_counts_into(text: Text, pattern: Pattern, out, ws, stream=None) -> None:
    """Enqueue one pm_crt_counts into caller-supplied tensors (out: n-m+1
    int32 counts, ws: crt_counts_workspace_bytes bytes)."""
    check(lib().pm_crt_counts(
        ctypes.c_void_p(text.data.data_ptr()), text.n, pattern.codes.ctypes.data, pattern.m,
        ctypes.c_void_p(out.data_ptr() if out.numel() else 0), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        _stream(stream)))


def scan_host_workspace_bytes(chunk_bases: int, m: int) -> int:
    return int(lib().pm_scan_host_workspace_bytes(int(chunk_bases), int(m)))


def scan_host(host_text, pattern: Pattern | str, k: int, chunk_bases: int = 1 << 27, capacity: int = 1 << 16,
              device=None, stream=None, copy_stream=None):
    """Scan a text that stays in host memory (a uint8 numpy array or CPU
    tensor of ASCII bases; pinned memory, e.g. torch.empty(..., pin_memory=
    True), copies fastest), streamed through the device in chunks of
    `chunk_bases` windows.  Returns (positions int64, counts uint16) device
    tensors equal to scan() of the encoded text; re-runs with an exact
    buffer when the hits exceed `capacity`."""
    import torch

    if isinstance(pattern, str):
        pattern = Pattern(pattern)
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    if isinstance(host_text, torch.Tensor):
        if host_text.device.type != "cpu" or host_text.dtype != torch.uint8 or not host_text.is_contiguous():
            raise ValueError("host_text must be a contiguous uint8 CPU tensor")
        ptr, n = host_text.data_ptr(), host_text.numel()
    else:
        host_text = np.ascontiguousarray(host_text, dtype=np.uint8)
        ptr, n = host_text.ctypes.data, host_text.size
    chunk_bases = max(1, min(int(chunk_bases), n))
    stream = stream or torch.cuda.current_stream(dev)
    copy_stream = copy_stream or torch.cuda.Stream(dev)
    ws = torch.empty(scan_host_workspace_bytes(chunk_bases, pattern.m), dtype=torch.uint8, device=dev)
    img = pattern.image(dev)
    n_hits = torch.zeros(1, dtype=torch.int64, device=dev)
    while True:
        pos = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
        cnt = torch.empty(max(capacity, 1), dtype=torch.uint16, device=dev)
        check(lib().pm_scan_host(
            ctypes.c_void_p(ptr), n, pattern.codes.ctypes.data, pattern.m, int(k), ctypes.c_void_p(img.data_ptr()),
            int(chunk_bases), ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), int(capacity),
            ctypes.c_void_p(n_hits.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
            _stream(stream), _stream(copy_stream)))
        total = int(n_hits.item())
        if total <= capacity:
            return pos[:total], cnt[:total]
        capacity = total


def scan(text: Text, pattern: Pattern | str, k: int, win_begin: int = 0, win_end: int | None = None,
         capacity: int = 1 << 16, ws: Workspace | None = None, stream=None):
    """All windows with at most k mismatches: (positions int64, counts uint16)
    as device tensors, ascending.  Re-runs with an exact buffer when the
    hits exceed `capacity`."""
    import torch

    if isinstance(pattern, str):
        pattern = Pattern(pattern)
    if ws is None:
        ws = Workspace(text.data.device, text.n, capacity)
    scan_async(text, pattern, k, ws, win_begin, win_end, stream)
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    total = int(ws.n_hits.item())
    if total > ws.capacity:
        ws.resize(total)
        scan_async(text, pattern, k, ws, win_begin, win_end, stream)
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        total = int(ws.n_hits.item())
    return ws.pos[:total].clone(), ws.cnt[:total].clone()


# --- FASTA input -----------------------------------------------------------------

class Fasta:
    """A parsed FASTA file (pm_fasta_parse): records, their bases
    concatenated (unknown bases written as 'A'), and the runs of unknown
    bases.  The scan reports only windows inside one record that cover no
    unknown base; positions are offsets in the concatenation."""

    def __init__(self, data: bytes | str):
        if isinstance(data, str):
            data = data.encode("ascii")
        h = ctypes.c_void_p()
        check(lib().pm_fasta_parse(data, len(data), ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_file(cls, path: str) -> "Fasta":
        with open(path, "rb") as f:
            return cls(f.read())

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.pm_fasta_free(self._h)
            self._h = ctypes.c_void_p()

    @property
    def n(self) -> int:
        return int(lib().pm_fasta_length(self._h))

    def bases(self) -> np.ndarray:
        """The concatenated bases (uint8 ASCII, a copy)."""
        n = self.n
        if n == 0:
            return np.zeros(0, dtype=np.uint8)
        ptr = lib().pm_fasta_bases(self._h)
        return np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(ptr)).copy()

    def records(self) -> list:
        """[(name, offset, length)] per record."""
        out = []
        for i in range(int(lib().pm_fasta_record_count(self._h))):
            name = ctypes.c_char_p()
            off, ln = ctypes.c_uint64(), ctypes.c_uint64()
            check(lib().pm_fasta_record(self._h, i, ctypes.byref(name), ctypes.byref(off), ctypes.byref(ln)))
            out.append((name.value.decode(), off.value, ln.value))
        return out

    def unknown_runs(self) -> list:
        """[(offset, length)] of the maximal runs of unknown bases."""
        out = []
        for i in range(int(lib().pm_fasta_unknown_run_count(self._h))):
            s, ln = ctypes.c_uint64(), ctypes.c_uint64()
            check(lib().pm_fasta_unknown_run(self._h, i, ctypes.byref(s), ctypes.byref(ln)))
            out.append((s.value, ln.value))
        return out

    def window_ranges(self, m: int) -> list:
        count = ctypes.c_uint64()
        check(lib().pm_fasta_window_ranges(self._h, int(m), None, None, 0, ctypes.byref(count)))
        b = np.zeros(max(count.value, 1), dtype=np.uint64)
        e = np.zeros(max(count.value, 1), dtype=np.uint64)
        check(lib().pm_fasta_window_ranges(self._h, int(m), b.ctypes.data, e.ctypes.data, count.value,
                                           ctypes.byref(count)))
        return list(zip(b[:count.value].tolist(), e[:count.value].tolist()))

    def encode(self, device=None, stream=None) -> Text:
        """The concatenated bases encoded in device memory (pm_encode_text)."""
        return encode_text(self.bases(), device=device, stream=stream)


def scan_fasta(fa: Fasta, text: Text, pattern: Pattern | str, k: int, capacity: int = 1 << 16, stream=None):
    """pm_scan_fasta: (positions int64, counts uint16) device tensors of the
    windows inside one record, covering no unknown base, with at most k
    mismatches; re-runs with an exact buffer when the hits exceed capacity."""
    import torch

    if isinstance(pattern, str):
        pattern = Pattern(pattern)
    dev = text.data.device
    img = pattern.image(dev)
    ws = torch.empty(int(lib().pm_scan_fasta_workspace_bytes(fa._h)), dtype=torch.uint8, device=dev)
    total = ctypes.c_uint64()
    while True:
        pos = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
        cnt = torch.empty(max(capacity, 1), dtype=torch.uint16, device=dev)
        check(lib().pm_scan_fasta(fa._h, ctypes.c_void_p(text.data.data_ptr()), pattern.codes.ctypes.data,
                                  pattern.m, int(k), ctypes.c_void_p(img.data_ptr()),
                                  ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), int(capacity),
                                  ctypes.byref(total), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
        if total.value <= capacity:
            return pos[:total.value], cnt[:total.value]
        capacity = int(total.value)


# --- batched scan ----------------------------------------------------------------

class BatchConfig(ctypes.Structure):
    """pm_batch_config: patterns per text tile, sub-ranges, lane words."""
    _fields_ = [("group_size", ctypes.c_uint32), ("sub_ranges", ctypes.c_uint32),
                ("lane_words", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def expected_hits(pattern: "Pattern", k: int, n: int) -> float:
    out = ctypes.c_double(0.0)
    check(lib().pm_expected_hits(pattern.codes.ctypes.data, pattern.m, int(k), int(n), ctypes.byref(out)))
    return out.value


def default_capacity(pattern: "Pattern", k: int, n: int) -> int:
    """Output slots for a pattern: twice the expected hits plus a margin."""
    return int(2 * expected_hits(pattern, k, n)) + 64


class Batch:
    """Host arrays of a batch of patterns (codes, lengths, budgets, capacities)."""

    def __init__(self, patterns, ks, n: int, capacities=None):
        self.patterns = [p if isinstance(p, Pattern) else Pattern(p) for p in patterns]
        self.ks = np.ascontiguousarray(ks, dtype=np.uint32)
        if self.ks.size != len(self.patterns):
            raise PMError(-1, "one k per pattern")
        self.m = np.array([p.m for p in self.patterns], dtype=np.uint32)
        self.codes = np.ascontiguousarray(np.concatenate([p.codes for p in self.patterns]), dtype=np.uint8)
        if capacities is None:
            capacities = [default_capacity(p, k, n) for p, k in zip(self.patterns, self.ks)]
        self.capacity = np.ascontiguousarray(capacities, dtype=np.uint64)
        self.out_off = np.zeros(len(self.patterns), dtype=np.uint64)
        if len(self.patterns) > 1:
            self.out_off[1:] = np.cumsum(self.capacity)[:-1]
        self.total_capacity = int(self.capacity.sum())

    def __len__(self):
        return len(self.patterns)


def batch_workspace_bytes(n: int, batch: Batch, config: BatchConfig | None = None) -> int:
    return int(lib().pm_scan_batch_workspace_bytes(
        n, len(batch), batch.m.ctypes.data, batch.capacity.ctypes.data,
        ctypes.byref(config) if config is not None else None))


def scan_batch_async(text: Text, batch: Batch, pos, cnt, n_hits, status, ws, win_begin: int = 0,
                     win_end: int | None = None, config: BatchConfig | None = None, stream=None) -> None:
    """Enqueue one pm_scan_batch; outputs are device tensors supplied by the caller."""
    if win_end is None:
        win_end = UINT64_MAX
    check(lib().pm_scan_batch(
        ctypes.c_void_p(text.data.data_ptr()), text.n, len(batch), batch.codes.ctypes.data,
        batch.m.ctypes.data, batch.ks.ctypes.data, batch.out_off.ctypes.data, batch.capacity.ctypes.data,
        int(win_begin), int(win_end), ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
        ctypes.c_void_p(n_hits.data_ptr()), ctypes.c_void_p(status.data_ptr()),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        ctypes.byref(config) if config is not None else None, _stream(stream)))


def scan_batch(text: Text, patterns, ks, capacities=None, config: BatchConfig | None = None,
               stream=None, rerun: bool = True):
    """Scan many patterns in one batched launch.  Returns a list of
    (positions, counts) device tensors, one per pattern, each complete: a
    pattern whose hits did not fit its share of the output is scanned again
    alone with an exact buffer (unless rerun=False, then it is None)."""
    import torch

    batch = patterns if isinstance(patterns, Batch) else Batch(patterns, ks, text.n, capacities)
    dev = text.data.device
    pos = torch.empty(max(batch.total_capacity, 1), dtype=torch.int64, device=dev)
    cnt = torch.empty(max(batch.total_capacity, 1), dtype=torch.uint16, device=dev)
    n_hits = torch.zeros(len(batch), dtype=torch.int64, device=dev)
    status = torch.zeros(len(batch), dtype=torch.int32, device=dev)
    ws = torch.empty(batch_workspace_bytes(text.n, batch, config), dtype=torch.uint8, device=dev)
    scan_batch_async(text, batch, pos, cnt, n_hits, status, ws, config=config, stream=stream)
    (torch.cuda.current_stream() if stream is None else stream).synchronize()
    nh = n_hits.cpu().numpy()
    st = status.cpu().numpy()
    out = []
    for i in range(len(batch)):
        if st[i] == 0:
            o = int(batch.out_off[i])
            out.append((pos[o:o + int(nh[i])], cnt[o:o + int(nh[i])]))
        elif rerun:
            out.append(scan(text, batch.patterns[i], int(batch.ks[i]), capacity=int(nh[i]) + 1,
                            stream=stream))
        else:
            out.append(None)
    return out
