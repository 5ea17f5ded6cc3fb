"""ctypes binding of ``libbpida.so`` (the C ABI declared in ``include/bpida.h``).

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  Importing this module loads the library and raises if it has not
been built; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

MAX_THRESHOLDS = 64
MAX_PATH = 256  # BPIDA_MAX_PATH
NOALLOC_SCRATCH_BYTES = 128 << 20  # BPIDA_NOALLOC_SCRATCH_BYTES
OK, EINVAL, EUNSOLVABLE, ELIMIT, ENOMEM, EDEVICE, EINTERNAL, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbpida.so")

EXPORTS = ("bpida_solve", "bpida_solve_paths", "bpida_solve_paths_device", "bpida_solve_mixed",
           "bpida_solve_mixed_device", "bpida_solve_device",
           "bpida_solve_device_async", "bpida_solve_device_noalloc", "bpida_set_option",
           "bpida_get_option", "bpida_last_stats", "bpida_strerror", "bpida_server_start",
           "bpida_server_submit", "bpida_server_poll", "bpida_server_stop")


class BpidaError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what or "bpida", strerror(code), code))


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbpida.so is not built; run `python -m paper_1705_02843_amd.build` "
                          "(or __graft_entry__.build())")
    # PyTorch ships its own HIP runtime, which its libraries load under a
    # name the dynamic linker does not match against an already loaded
    # ROCm copy: loading libbpida.so (which needs libamdhip64.so.7) first
    # would leave two HIP runtimes in the process, and torch's device copies
    # then crash.  Importing torch first makes the library bind to torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.bpida_solve.argtypes = [P(ctypes.c_uint8), ctypes.c_int32, ctypes.c_int32,
                                P(ctypes.c_int32), P(ctypes.c_uint64)]
    lib.bpida_solve.restype = ctypes.c_int
    lib.bpida_solve_paths.argtypes = [P(ctypes.c_uint8), ctypes.c_int32, ctypes.c_int32,
                                      P(ctypes.c_int32), P(ctypes.c_uint64), P(ctypes.c_uint8)]
    lib.bpida_solve_paths.restype = ctypes.c_int
    lib.bpida_solve_paths_device.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
    lib.bpida_solve_paths_device.restype = ctypes.c_int
    lib.bpida_solve_mixed.argtypes = [P(ctypes.c_uint8), P(ctypes.c_int32), ctypes.c_int32,
                                      P(ctypes.c_int32), P(ctypes.c_uint64)]
    lib.bpida_solve_mixed.restype = ctypes.c_int
    lib.bpida_solve_mixed_device.argtypes = [ctypes.c_void_p, P(ctypes.c_int32), ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.bpida_solve_mixed_device.restype = ctypes.c_int
    lib.bpida_solve_device.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.bpida_solve_device.restype = ctypes.c_int
    lib.bpida_solve_device_async.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
    lib.bpida_solve_device_async.restype = ctypes.c_int
    lib.bpida_solve_device_noalloc.argtypes = lib.bpida_solve_device_async.argtypes
    lib.bpida_solve_device_noalloc.restype = ctypes.c_int
    lib.bpida_server_start.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p]
    lib.bpida_server_start.restype = ctypes.c_int
    lib.bpida_server_submit.argtypes = [P(ctypes.c_uint8), P(ctypes.c_uint64)]
    lib.bpida_server_submit.restype = ctypes.c_int
    lib.bpida_server_poll.argtypes = [ctypes.c_uint64, P(ctypes.c_int32), P(ctypes.c_uint64),
                                      P(ctypes.c_int32)]
    lib.bpida_server_poll.restype = ctypes.c_int
    lib.bpida_server_stop.argtypes = []
    lib.bpida_server_stop.restype = ctypes.c_int
    lib.bpida_set_option.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    lib.bpida_set_option.restype = ctypes.c_int
    lib.bpida_get_option.argtypes = [ctypes.c_char_p]
    lib.bpida_get_option.restype = ctypes.c_int64
    lib.bpida_last_stats.argtypes = [P(ctypes.c_uint64), ctypes.c_int32]
    lib.bpida_last_stats.restype = ctypes.c_int
    lib.bpida_strerror.argtypes = [ctypes.c_int]
    lib.bpida_strerror.restype = ctypes.c_char_p
    return lib


lib = _load()


def strerror(code: int) -> str:
    return lib.bpida_strerror(int(code)).decode()


def set_option(key: str, value: int) -> None:
    rc = lib.bpida_set_option(key.encode(), int(value))
    if rc != OK:
        raise BpidaError(rc, "set_option(%s=%r)" % (key, value))


def get_option(key: str) -> int:
    return int(lib.bpida_get_option(key.encode()))


def last_stats() -> dict:
    out = (ctypes.c_uint64 * 20)()
    rc = lib.bpida_last_stats(out, 20)
    if rc != OK:
        raise BpidaError(rc, "last_stats")
    keys = ("rounds", "search_nodes", "spilled", "launches", "search_us", "spill_high_water",
            "chunks_pushed", "chunks_popped", "wg_us_search", "wg_us_queue", "wg_us_idle",
            "donations_voluntary", "grid", "error_bits", "queue_slots", "lb_roots_added",
            "roots_read", "wide_chunks_taken")
    return {k: int(out[i]) for i, k in enumerate(keys)}


def solve_raw(states: np.ndarray, width: int = 4):
    """Host-buffer entry point.  Returns (rc, out_len int32[n], nodes uint64[n, 64])."""
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint8).reshape(-1, width * width))
    n = st.shape[0]
    out_len = np.full(n, -7, np.int32)
    nodes = np.zeros((n, MAX_THRESHOLDS), np.uint64)
    rc = lib.bpida_solve(st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), n, width,
                         out_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return int(rc), out_len, nodes


def solve_paths_raw(states: np.ndarray, width: int = 4):
    """Host-buffer entry with paths.  Returns (rc, out_len int32[n],
    nodes uint64[n, 64], path uint8[n, 256]: moves U, L, R, D = 0..3, 0xFF
    past the length)."""
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint8).reshape(-1, width * width))
    n = st.shape[0]
    out_len = np.full(n, -7, np.int32)
    nodes = np.zeros((n, MAX_THRESHOLDS), np.uint64)
    path = np.zeros((n, MAX_PATH), np.uint8)
    rc = lib.bpida_solve_paths(st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), n, width,
                               out_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               path.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return int(rc), out_len, nodes, path


def solve_paths_device(d_states, d_len, d_nodes, d_path, width: int = 4, stream=None) -> int:
    """Device-buffer entry with paths on torch tensors (as ``solve_device``,
    plus ``d_path`` uint8 [n, 256])."""
    import torch  # device buffers and streams only

    n = int(d_states.shape[0])
    assert d_states.is_cuda and d_states.dtype == torch.uint8 and d_states.is_contiguous()
    assert d_states.numel() == n * width * width
    assert d_len.is_cuda and d_len.dtype == torch.int32 and d_len.numel() >= n
    assert d_nodes.is_cuda and d_nodes.dtype in (torch.int64, torch.uint64)
    assert d_nodes.is_contiguous() and d_nodes.numel() >= n * MAX_THRESHOLDS
    assert d_path.is_cuda and d_path.dtype == torch.uint8 and d_path.is_contiguous()
    assert d_path.numel() >= n * MAX_PATH
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(lib.bpida_solve_paths_device(ctypes.c_void_p(d_states.data_ptr()), n, width,
                                            ctypes.c_void_p(d_len.data_ptr()),
                                            ctypes.c_void_p(d_nodes.data_ptr()),
                                            ctypes.c_void_p(d_path.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream)))


def solve_mixed_raw(states_list):
    """Batch of states of mixed widths (a list of uint8 vectors of w*w
    entries).  Returns (rc, out_len int32[n], nodes uint64[n, 64])."""
    widths = np.array([int(round(len(s) ** 0.5)) for s in states_list], np.int32)
    for k, (s, w) in enumerate(zip(states_list, widths)):
        if len(s) != int(w) * int(w):
            raise ValueError("state %d has %d entries, not a square board" % (k, len(s)))
    flat = np.ascontiguousarray(np.concatenate([np.asarray(s, np.uint8).reshape(-1)
                                                for s in states_list]) if states_list
                                else np.zeros(0, np.uint8))
    n = len(states_list)
    out_len = np.full(n, -7, np.int32)
    nodes = np.zeros((n, MAX_THRESHOLDS), np.uint64)
    rc = lib.bpida_solve_mixed(flat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                               widths.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n,
                               out_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return int(rc), out_len, nodes


def solve(states, width: int = 4):
    """Solve a batch given as a numpy array; raises BpidaError on failure."""
    rc, out_len, nodes = solve_raw(states, width)
    if rc != OK:
        raise BpidaError(rc, "bpida_solve")
    return out_len, nodes


def solve_device(d_states, d_len, d_nodes, width: int = 4, stream=None) -> int:
    """Device-buffer entry point on torch tensors (uint8 [n, w*w], int32 [n],
    int64/uint64 [n, 64]) of the current device.  ``stream`` is a
    ``torch.cuda.Stream`` (default: torch's current stream).  Returns the
    status code."""
    import torch  # device buffers and streams only

    n = int(d_states.shape[0])
    assert d_states.is_cuda and d_states.dtype == torch.uint8 and d_states.is_contiguous()
    assert d_states.numel() == n * width * width
    assert d_len.is_cuda and d_len.dtype == torch.int32 and d_len.numel() >= n
    assert d_nodes.is_cuda and d_nodes.dtype in (torch.int64, torch.uint64)
    assert d_nodes.is_contiguous() and d_nodes.numel() >= n * MAX_THRESHOLDS
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(lib.bpida_solve_device(ctypes.c_void_p(d_states.data_ptr()), n, width,
                                      ctypes.c_void_p(d_len.data_ptr()),
                                      ctypes.c_void_p(d_nodes.data_ptr()),
                                      ctypes.c_void_p(s.cuda_stream)))


def solve_mixed_device(d_states, widths, d_len, d_nodes, stream=None) -> int:
    """Mixed-width batch on torch tensors: ``d_states`` uint8 on the device,
    the instances' bytes back to back; ``widths`` host int32 [n] (numpy).
    Outputs as in ``solve_device``.  Returns the status code."""
    import torch  # device buffers and streams only

    w = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    n = int(w.shape[0])
    assert d_states.is_cuda and d_states.dtype == torch.uint8 and d_states.is_contiguous()
    assert d_states.numel() == int((w.astype(np.int64) ** 2).sum())
    assert d_len.is_cuda and d_len.dtype == torch.int32 and d_len.numel() >= n
    assert d_nodes.is_cuda and d_nodes.dtype in (torch.int64, torch.uint64)
    assert d_nodes.is_contiguous() and d_nodes.numel() >= n * MAX_THRESHOLDS
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(lib.bpida_solve_mixed_device(ctypes.c_void_p(d_states.data_ptr()),
                                            w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n,
                                            ctypes.c_void_p(d_len.data_ptr()),
                                            ctypes.c_void_p(d_nodes.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream)))


def solve_device_async(d_states, d_len, d_nodes, d_status, width: int = 4, stream=None) -> int:
    """Enqueue a batched solve on torch tensors without waiting (capturable
    into a graph); per-instance status goes to ``d_status`` (int32 [n])."""
    import torch  # device buffers and streams only

    n = int(d_states.shape[0])
    assert d_states.is_cuda and d_states.dtype == torch.uint8 and d_states.is_contiguous()
    assert d_states.numel() == n * width * width
    assert d_len.is_cuda and d_len.dtype == torch.int32 and d_len.numel() >= n
    assert d_status.is_cuda and d_status.dtype == torch.int32 and d_status.numel() >= n
    assert d_nodes.is_cuda and d_nodes.dtype in (torch.int64, torch.uint64)
    assert d_nodes.is_contiguous() and d_nodes.numel() >= n * MAX_THRESHOLDS
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(lib.bpida_solve_device_async(ctypes.c_void_p(d_states.data_ptr()), n, width,
                                            ctypes.c_void_p(d_len.data_ptr()),
                                            ctypes.c_void_p(d_nodes.data_ptr()),
                                            ctypes.c_void_p(d_status.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream)))


def solve_device_noalloc(d_states, d_len, d_nodes, d_status, width: int = 4, stream=None) -> int:
    """As ``solve_device_async`` through the entry point that allocates no
    device memory (its buffers come from a fixed array inside the library)."""
    import torch  # device buffers and streams only

    n = int(d_states.shape[0])
    assert d_states.is_cuda and d_states.dtype == torch.uint8 and d_states.is_contiguous()
    assert d_states.numel() == n * width * width
    assert d_len.is_cuda and d_len.dtype == torch.int32 and d_len.numel() >= n
    assert d_status.is_cuda and d_status.dtype == torch.int32 and d_status.numel() >= n
    assert d_nodes.is_cuda and d_nodes.dtype in (torch.int64, torch.uint64)
    assert d_nodes.is_contiguous() and d_nodes.numel() >= n * MAX_THRESHOLDS
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(lib.bpida_solve_device_noalloc(ctypes.c_void_p(d_states.data_ptr()), n, width,
                                              ctypes.c_void_p(d_len.data_ptr()),
                                              ctypes.c_void_p(d_nodes.data_ptr()),
                                              ctypes.c_void_p(d_status.data_ptr()),
                                              ctypes.c_void_p(s.cuda_stream)))


class Server:
    """Continuous-batching server on the C ABI (one per process)."""

    def __init__(self, max_inflight: int = 512, ring_capacity: int = 4096, width: int = 4):
        self.width = width
        rc = lib.bpida_server_start(width, max_inflight, ring_capacity, None)
        if rc != OK:
            raise BpidaError(rc, "bpida_server_start")
        self.running = True

    def submit(self, state) -> int | None:
        """Queue one state; returns its ticket, or None if the ring is full."""
        st = np.ascontiguousarray(np.asarray(state, dtype=np.uint8).reshape(-1))
        t = ctypes.c_uint64(0)
        rc = lib.bpida_server_submit(st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                     ctypes.byref(t))
        if rc == EAGAIN:
            return None
        if rc != OK:
            raise BpidaError(rc, "bpida_server_submit")
        return int(t.value)

    def poll(self, ticket: int):
        """(length, nodes uint64[64], status) once answered, else None."""
        ln = ctypes.c_int32(0)
        stt = ctypes.c_int32(0)
        nodes = np.zeros(MAX_THRESHOLDS, np.uint64)
        rc = lib.bpida_server_poll(ticket, ctypes.byref(ln),
                                   nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   ctypes.byref(stt))
        if rc == 0:
            return None
        if rc != 1:
            raise BpidaError(rc, "bpida_server_poll")
        return int(ln.value), nodes, int(stt.value)

    def stop(self) -> int:
        if not self.running:
            return OK
        self.running = False
        return int(lib.bpida_server_stop())

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
