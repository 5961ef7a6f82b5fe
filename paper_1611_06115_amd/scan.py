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
