"""ctypes binding of the query server of libpmscan (pm_server_* in
include/pmscan.h): argument marshalling only.  The engine (admission, chunk
steps, joins) is native; torch provides the arena and the stream."""
from __future__ import annotations

import ctypes

import numpy as np

from .scan import BatchConfig, Pattern, PMError, Text, check, lib

WAITING, ACTIVE, DONE, FAILED = 0, 1, 2, 3


class ServerConfig(ctypes.Structure):
    """pm_server_config."""
    _fields_ = [("chunks", ctypes.c_uint32), ("max_active", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64), ("batch", BatchConfig)]


class QueryInfo(ctypes.Structure):
    """pm_query_info."""
    _fields_ = [("state", ctypes.c_int32), ("error", ctypes.c_int32), ("n_hits", ctypes.c_uint64),
                ("pos_dev", ctypes.c_void_p), ("cnt_dev", ctypes.c_void_p),
                ("arrival_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
                ("complete_ns", ctypes.c_uint64), ("first_chunk", ctypes.c_uint32),
                ("reruns", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    """pm_server_stats."""
    _fields_ = [("steps", ctypes.c_uint64), ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64), ("reruns", ctypes.c_uint64),
                ("comparisons", ctypes.c_uint64), ("active", ctypes.c_uint32), ("waiting", ctypes.c_uint32),
                ("peak_active", ctypes.c_uint32), ("chunks", ctypes.c_uint32), ("hit_slots", ctypes.c_uint64),
                ("hit_slots_used", ctypes.c_uint64), ("hit_slots_peak", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def now_ns() -> int:
    return int(lib().pm_server_now_ns())


def min_arena_bytes(n: int, config: ServerConfig | None = None) -> int:
    return int(lib().pm_server_min_arena_bytes(n, ctypes.byref(config) if config is not None else None))


class Server:
    """A query server over a resident encoded text.

    mem_budget: bytes of device memory for the arena (a torch tensor owned by
    this object).  The server keeps `text` alive; close() stops the engine."""

    def __init__(self, text: Text, mem_budget: int, config: ServerConfig | None = None, stream=None):
        import torch

        self.text = text
        dev = text.data.device
        self.config = config if config is not None else ServerConfig()
        self.arena = torch.empty(int(mem_budget), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self._h = ctypes.c_void_p()
        check(lib().pm_server_create(ctypes.c_void_p(text.data.data_ptr()), text.n,
                                     ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                     ctypes.byref(self.config), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(self._h)))

    def _handle(self):
        if not self._h:
            raise PMError(-1, "server is closed")
        return self._h

    def submit(self, pattern: Pattern | str | np.ndarray, k: int, arrival_ns: int = 0) -> int:
        if not isinstance(pattern, Pattern):
            pattern = Pattern(pattern)
        qid = ctypes.c_uint64(0)
        check(lib().pm_server_submit(self._handle(), pattern.codes.ctypes.data, pattern.m, int(k),
                                     int(arrival_ns), ctypes.byref(qid)))
        return int(qid.value)

    def poll(self, qid: int) -> QueryInfo:
        info = QueryInfo()
        check(lib().pm_server_poll(self._handle(), int(qid), ctypes.byref(info)))
        return info

    def wait(self, qid: int, timeout_ms: int = -1) -> QueryInfo:
        info = QueryInfo()
        check(lib().pm_server_wait(self._handle(), int(qid), int(timeout_ms), ctypes.byref(info)))
        return info

    def result(self, qid: int, release: bool = True, timeout_ms: int = -1):
        """Wait for a query and return (positions, counts) as new device tensors."""
        import torch

        info = self.wait(qid, timeout_ms)
        if info.state != DONE:
            raise PMError(int(info.error), f"query {qid} failed")
        n = int(info.n_hits)
        dev = self.arena.device
        pos = torch.empty(n, dtype=torch.int64, device=dev)
        cnt = torch.empty(n, dtype=torch.uint16, device=dev)
        if n:
            base = self.arena.data_ptr()
            o_pos = (int(info.pos_dev) - base) // 8
            o_cnt = (int(info.cnt_dev) - base) // 2
            if (int(info.pos_dev) - base) % 8 or (int(info.cnt_dev) - base) % 2:
                raise PMError(-1, "misaligned result")
            with torch.cuda.stream(self.stream):
                pos.copy_(self._view(torch.int64, o_pos, n))
                cnt.copy_(self._view(torch.uint16, o_cnt, n))
            self.stream.synchronize()
        if release:
            self.release(qid)
        return pos, cnt

    def _view(self, dtype, offset, n):
        import torch

        size = torch.tensor([], dtype=dtype).element_size()
        usable = self.arena.numel() // size * size
        return self.arena[:usable].view(dtype)[offset:offset + n]

    def release(self, qid: int) -> None:
        check(lib().pm_server_release(self._handle(), int(qid)))

    def drain(self, timeout_ms: int = -1) -> None:
        check(lib().pm_server_drain(self._handle(), int(timeout_ms)))

    def stats(self) -> dict:
        s = ServerStats()
        check(lib().pm_server_stats_get(self._handle(), ctypes.byref(s)))
        return s.as_dict()

    def error_detail(self) -> str:
        return lib().pm_server_error_detail(self._handle()).decode()

    def close(self) -> None:
        if self._h:
            check(lib().pm_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
