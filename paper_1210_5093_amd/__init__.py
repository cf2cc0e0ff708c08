"""MI355X speculative DFA membership test (arXiv 1210.5093) -- Python binding.

Thin ctypes layer over ``libdfaspec.so`` (``include/dfa_spec.h``): argument
marshalling only.  Every step of the matching runs in the library's HIP
kernels; there is no Python or CPU fallback, and loading fails loudly if the
library has not been built.  torch is used only for device buffers and
stream handles.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfaspec.so")

DFA_OK = 0
DFA_E_INVAL, DFA_E_NOMEM, DFA_E_DEVICE, DFA_E_SYMBOL = -1, -2, -3, -4
DFA_E_TOOBIG, DFA_E_SPECULATION, DFA_E_BUSY, DFA_E_NOTREADY = -5, -6, -7, -8
DFA_Q0 = 0xFFFFFFFF
DFA_LOOKAHEAD_AUTO = 0xFFFFFFFF
FLAG_SYMBOL, FLAG_SPECULATION = 1, 2


class DFAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class dfa_info_t(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_uint32), ("num_symbols", ctypes.c_uint32),
                ("num_classes", ctypes.c_uint32), ("num_absorbing", ctypes.c_uint32),
                ("imax", ctypes.c_uint32), ("q0", ctypes.c_uint32),
                ("mean_iset", ctypes.c_double), ("table_bytes", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("packed_layout", ctypes.c_uint32),
                ("lookahead_tables", ctypes.c_uint32), ("pair_columns", ctypes.c_uint32)]


class dfa_match_opts_t(ctypes.Structure):
    _fields_ = [("chunk_len", ctypes.c_uint64), ("lookahead", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class dfa_plan_info_t(ctypes.Structure):
    _fields_ = [("chunk_len", ctypes.c_uint64), ("num_chunks", ctypes.c_uint64),
                ("kernel", ctypes.c_uint32), ("lookahead", ctypes.c_uint32),
                ("blocks", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("symbols_per_step", ctypes.c_uint32), ("raw_input", ctypes.c_uint32),
                ("rounds", ctypes.c_uint32), ("interleaved", ctypes.c_uint32),
                ("chunk_lanes", ctypes.c_uint32), ("set_max", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("group0", ctypes.c_uint32),
                ("group", ctypes.c_uint32), ("tail_lanes", ctypes.c_uint32),
                ("tail_start", ctypes.c_uint32)]


class dfa_result_t(ctypes.Structure):
    _fields_ = [("final_state", ctypes.c_uint32), ("accepted", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("num_chunks", ctypes.c_uint32)]


class dfa_server_done_t(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("result", dfa_result_t),
                ("submit_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64)]


class dfa_server_opts_t(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("lookahead", ctypes.c_uint32), ("slot_bytes", ctypes.c_uint64)]


class dfa_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("inflight", ctypes.c_uint64), ("pending", ctypes.c_uint64)]


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libdfaspec.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(the HIP library is required, there is no fallback)")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # loading torch first makes the library bind to that one copy, so device
    # pointers and streams are shared within the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.dfa_create.restype = I
    L.dfa_create.argtypes = [P, U32, U32, U32, P, U32, P, ctypes.POINTER(P)]
    L.dfa_destroy.restype = None
    L.dfa_destroy.argtypes = [P]
    L.dfa_info.restype = I
    L.dfa_info.argtypes = [P, ctypes.POINTER(dfa_info_t)]
    L.dfa_match.restype = I
    L.dfa_match.argtypes = [P, P, ctypes.c_size_t, U32, ctypes.POINTER(U32),
                            ctypes.POINTER(ctypes.c_int)]
    L.dfa_match_async.restype = I
    L.dfa_match_async.argtypes = [P, P, ctypes.c_size_t, U32, P, P]
    L.dfa_match_ex.restype = I
    L.dfa_match_ex.argtypes = [P, P, ctypes.c_size_t, U32, ctypes.POINTER(dfa_match_opts_t), P,
                               P, P]
    L.dfa_match_noalloc.restype = I
    L.dfa_match_noalloc.argtypes = [P, P, ctypes.c_size_t, U32,
                                    ctypes.POINTER(dfa_match_opts_t), P, P, P]
    L.dfa_match_maps.restype = I
    L.dfa_match_maps.argtypes = [P, P, ctypes.c_size_t, U32, ctypes.POINTER(dfa_match_opts_t), P,
                                 P, P, P, P, U64]
    L.dfa_plan_chunks.restype = I
    L.dfa_plan_chunks.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(dfa_match_opts_t),
                                  ctypes.POINTER(U64), ctypes.POINTER(U64)]
    L.dfa_lookahead_set.restype = I
    L.dfa_lookahead_set.argtypes = [P, P, U32, P, U32, ctypes.POINTER(U32)]
    L.dfa_plan.restype = I
    L.dfa_plan.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(dfa_match_opts_t),
                           ctypes.POINTER(dfa_plan_info_t)]
    L.dfa_batch_create.restype = I
    L.dfa_batch_create.argtypes = [P, P, P, ctypes.c_size_t, ctypes.POINTER(dfa_match_opts_t),
                                   ctypes.POINTER(P)]
    L.dfa_batch_run.restype = I
    L.dfa_batch_run.argtypes = [P, P, P]
    L.dfa_batch_graph_launch.restype = I
    L.dfa_batch_graph_launch.argtypes = [P, P, P]
    L.dfa_batch_info.restype = I
    L.dfa_batch_info.argtypes = [P, ctypes.POINTER(U64), ctypes.POINTER(U32)]
    L.dfa_batch_destroy.restype = None
    L.dfa_batch_destroy.argtypes = [P]
    L.dfa_server_drain.restype = I
    L.dfa_server_drain.argtypes = [P, ctypes.POINTER(dfa_server_done_t), ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_size_t)]
    L.dfa_autotune.restype = I
    L.dfa_autotune.argtypes = [P, P, ctypes.c_size_t, P, ctypes.POINTER(dfa_match_opts_t),
                               ctypes.POINTER(ctypes.c_double)]
    L.dfa_batch_tune.restype = I
    L.dfa_batch_tune.argtypes = [P, P, P, ctypes.c_size_t, P, ctypes.POINTER(dfa_match_opts_t),
                                 ctypes.POINTER(ctypes.c_double)]
    L.dfa_server_create.restype = I
    L.dfa_server_create.argtypes = [ctypes.POINTER(dfa_server_opts_t), ctypes.POINTER(P)]
    L.dfa_server_register.restype = I
    L.dfa_server_register.argtypes = [P, P, ctypes.POINTER(U32)]
    L.dfa_server_submit.restype = I
    L.dfa_server_submit.argtypes = [P, U32, P, ctypes.c_size_t, ctypes.POINTER(U64)]
    L.dfa_server_submit_after.restype = I
    L.dfa_server_submit_after.argtypes = [P, U32, P, ctypes.c_size_t, P, ctypes.POINTER(U64)]
    L.dfa_server_poll.restype = I
    L.dfa_server_poll.argtypes = [P, U64, ctypes.POINTER(dfa_result_t)]
    L.dfa_server_wait.restype = I
    L.dfa_server_wait.argtypes = [P, U64, ctypes.POINTER(dfa_result_t)]
    L.dfa_server_stats.restype = I
    L.dfa_server_stats.argtypes = [P, ctypes.POINTER(dfa_server_stats_t)]
    L.dfa_server_destroy.restype = None
    L.dfa_server_destroy.argtypes = [P]
    L.dfa_match_batch.restype = I
    L.dfa_match_batch.argtypes = [P, P, P, ctypes.c_size_t, P, P]
    L.dfa_timing_enable.restype = I
    L.dfa_timing_enable.argtypes = [P, I]
    L.dfa_timing_read.restype = I
    L.dfa_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U32)]
    L.dfa_timing_read_ex.restype = I
    L.dfa_timing_read_ex.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U32)]
    L.dfa_match_block.restype = I
    L.dfa_match_block.argtypes = [P, P, ctypes.c_size_t, ctypes.c_size_t, U32,
                                  ctypes.POINTER(dfa_match_opts_t), P, P, P, P, U32]
    L.dfa_compose_blocks.restype = I
    L.dfa_compose_blocks.argtypes = [P, U32, P, P, P, U32, U32, P, P, P]
    L.dfa_strerror.restype = ctypes.c_char_p
    L.dfa_strerror.argtypes = [I]
    L.dfa_last_error.restype = ctypes.c_char_p
    L.dfa_last_error.argtypes = []
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != DFA_OK:
        raise DFAError(rc, lib().dfa_last_error().decode(errors="replace")
                       or lib().dfa_strerror(rc).decode())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


MATCH_EARLY_EXIT = 1
MATCH_SINGLE_STEP = 2
MATCH_INTERLEAVE = 4
MATCH_CHUNK_LANES = 8


def match_rounds(k: int) -> int:
    """flags bits of DFA_MATCH_ROUNDS(k): walk rounds with merging (0 = planner)."""
    return (int(k) & 0xF) << 8


def _opts(chunk_len: int = 0, lookahead: int = 1, early_exit: bool = False,
          rounds: int = 0, single_step: bool = False, interleave: bool = False,
          chunk_lanes: bool = False) -> dfa_match_opts_t:
    flags = ((MATCH_EARLY_EXIT if early_exit else 0) | match_rounds(rounds) |
             (MATCH_SINGLE_STEP if single_step else 0) | (MATCH_INTERLEAVE if interleave else 0) |
             (MATCH_CHUNK_LANES if chunk_lanes else 0))
    return dfa_match_opts_t(int(chunk_len), int(lookahead), flags)


class DFA:
    """A DFA (Q, Sigma, delta, q0, F) compiled and resident on the current device."""

    def __init__(self, delta, q0: int, accepting, byte_to_symbol=None):
        d = np.ascontiguousarray(delta, dtype=np.uint32)
        if d.ndim != 2:
            raise ValueError("delta must be a 2-D table [num_states][num_symbols]")
        acc = np.ascontiguousarray(accepting, dtype=np.uint32)
        b2s = None if byte_to_symbol is None else np.ascontiguousarray(byte_to_symbol,
                                                                       dtype=np.uint8)
        if b2s is not None and b2s.size != 256:
            raise ValueError("byte_to_symbol must have 256 entries")
        h = ctypes.c_void_p()
        _check(lib().dfa_create(d.ctypes.data, d.shape[0], d.shape[1], int(q0),
                                acc.ctypes.data if acc.size else None, int(acc.size),
                                b2s.ctypes.data if b2s is not None else None, ctypes.byref(h)))
        self._h = h
        self.num_states, self.num_symbols = int(d.shape[0]), int(d.shape[1])

    @classmethod
    def from_workload(cls, w) -> "DFA":
        return cls(w.delta, w.q0, w.accepting, w.byte_to_symbol)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("DFA was destroyed")
        return self._h

    def info(self) -> dfa_info_t:
        out = dfa_info_t()
        _check(lib().dfa_info(self.handle, ctypes.byref(out)))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().dfa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dfa_create(delta, q0, accepting, byte_to_symbol=None) -> DFA:
    return DFA(delta, q0, accepting, byte_to_symbol)


def dfa_match(d: DFA, data, start: Optional[int] = None) -> Tuple[int, bool]:
    """Synchronous test of host bytes: (final state, accepted)."""
    buf = np.frombuffer(bytes(data), dtype=np.uint8) if isinstance(data, (bytes, bytearray)) \
        else np.ascontiguousarray(data, dtype=np.uint8)
    fin = ctypes.c_uint32()
    acc = ctypes.c_int()
    _check(lib().dfa_match(d.handle, buf.ctypes.data if buf.size else None, int(buf.size),
                           DFA_Q0 if start is None else int(start), ctypes.byref(fin),
                           ctypes.byref(acc)))
    return int(fin.value), bool(acc.value)


def _result_tensor(result):
    import torch
    if result is None:
        result = torch.empty(4, dtype=torch.int32, device="cuda")
    assert result.is_cuda and result.dtype in (torch.int32, torch.uint32) and result.numel() >= 4
    return result


def dfa_match_async(d: DFA, d_input, start: Optional[int] = None, stream=None, result=None):
    """Enqueue the test of a device uint8 tensor; returns the 4-int32 result tensor
    (final, accepted, flags, num_chunks) written on the stream."""
    result = _result_tensor(result)
    _check(lib().dfa_match_async(d.handle, d_input.data_ptr() if d_input.numel() else None,
                                 int(d_input.numel()), DFA_Q0 if start is None else int(start),
                                 _stream_handle(stream), result.data_ptr()))
    return result


def dfa_plan_chunks(d: DFA, n: int, chunk_len: int = 0, lookahead: int = 1) -> Tuple[int, int]:
    c, k = ctypes.c_uint64(), ctypes.c_uint64()
    o = _opts(chunk_len, lookahead)
    _check(lib().dfa_plan_chunks(d.handle, int(n), ctypes.byref(o), ctypes.byref(c),
                                 ctypes.byref(k)))
    return int(c.value), int(k.value)


def dfa_lookahead_set(d: DFA, lookahead_bytes) -> List[int]:
    """Precomputed initial-state set for k lookahead bytes (Eq. 13)."""
    b = np.frombuffer(bytes(lookahead_bytes), dtype=np.uint8)
    out = np.zeros(d.num_states, dtype=np.uint16)
    cnt = ctypes.c_uint32()
    _check(lib().dfa_lookahead_set(d.handle, b.ctypes.data, int(b.size), out.ctypes.data,
                                   int(out.size), ctypes.byref(cnt)))
    return out[:cnt.value].tolist()


def dfa_plan(d: DFA, n: int, chunk_len: int = 0, lookahead: int = 1, rounds: int = 0,
             early_exit: bool = False, single_step: bool = False,
             interleave: bool = False, chunk_lanes: bool = False) -> dfa_plan_info_t:
    out = dfa_plan_info_t()
    o = _opts(chunk_len, lookahead, early_exit, rounds, single_step, interleave, chunk_lanes)
    _check(lib().dfa_plan(d.handle, int(n), ctypes.byref(o), ctypes.byref(out)))
    return out


def dfa_match_ex(d: DFA, d_input, start: Optional[int] = None, chunk_len: int = 0,
                 lookahead: int = 1, boundaries: bool = False, stream=None, result=None,
                 bound_out=None, early_exit: bool = False, rounds: int = 0,
                 single_step: bool = False, interleave: bool = False, chunk_lanes: bool = False):
    """Test with options; optionally the state at every chunk boundary.
    rounds: walk rounds with merging (DFA_MATCH_ROUNDS; 0 = the planner's);
    single_step: one symbol per lookup even with a two-symbol table;
    interleave: chunk-interleaved code stream (else linear; direct tables: the raw input);
    chunk_lanes: one chunk per lane with merged walks.
    Returns (result tensor, boundaries tensor or None)."""
    import torch
    result = _result_tensor(result)
    n = int(d_input.numel())
    bnd = None
    if boundaries:
        _, nch = dfa_plan_chunks(d, n, chunk_len, lookahead)
        bnd = bound_out if bound_out is not None else torch.empty(
            nch + 1, dtype=torch.int32, device="cuda")
        assert bnd.numel() >= nch + 1
    o = _opts(chunk_len, lookahead, early_exit, rounds, single_step, interleave, chunk_lanes)
    _check(lib().dfa_match_ex(d.handle, d_input.data_ptr() if n else None, n,
                              DFA_Q0 if start is None else int(start), ctypes.byref(o),
                              _stream_handle(stream), result.data_ptr(),
                              bnd.data_ptr() if bnd is not None else None))
    return result, bnd


def dfa_match_noalloc(d: DFA, d_input, start: Optional[int] = None, chunk_len: int = 0,
                      lookahead: int = 1, boundaries: bool = False, stream=None, result=None,
                      bound_out=None, early_exit: bool = False, rounds: int = 0,
                      single_step: bool = False, interleave: bool = False,
                      chunk_lanes: bool = False):
    """dfa_match_noalloc: dfa_match_ex with every scratch buffer in the library's
    fixed per-GPU region (no device allocation by the library).  Returns
    (result tensor, boundaries tensor or None); pass `result` and `bound_out`
    to allocate nothing on the Python side either."""
    import torch
    result = _result_tensor(result)
    n = int(d_input.numel())
    bnd = None
    if boundaries:
        _, nch = dfa_plan_chunks(d, n, chunk_len, lookahead)
        bnd = bound_out if bound_out is not None else torch.empty(
            nch + 1, dtype=torch.int32, device="cuda")
        assert bnd.numel() >= nch + 1
    o = _opts(chunk_len, lookahead, early_exit, rounds, single_step, interleave, chunk_lanes)
    _check(lib().dfa_match_noalloc(d.handle, d_input.data_ptr() if n else None, n,
                                   DFA_Q0 if start is None else int(start), ctypes.byref(o),
                                   _stream_handle(stream), result.data_ptr(),
                                   bnd.data_ptr() if bnd is not None else None))
    return result, bnd


def dfa_match_maps(d: DFA, d_input, start: Optional[int] = None, chunk_len: int = 0,
                   lookahead: int = 1, stream=None, result=None, max_pairs: Optional[int] = None,
                   early_exit: bool = False, rounds: int = 0, single_step: bool = False,
                   interleave: bool = False, chunk_lanes: bool = False):
    """dfa_match_maps: the test plus its level-0 state maps.  Returns (result
    tensor, first [num_chunks + 1] int32, pair start states int16, pair end
    states int16), all device tensors; pair P of chunk i (first[i] <= P <
    first[i + 1]) walked chunk i from start[P] and ended in end[P]."""
    import torch
    result = _result_tensor(result)
    n = int(d_input.numel())
    o = _opts(chunk_len, lookahead, early_exit, rounds, single_step, interleave, chunk_lanes)
    plan = dfa_plan_info_t()
    _check(lib().dfa_plan(d.handle, n, ctypes.byref(o), ctypes.byref(plan)))
    nch = int(plan.num_chunks)
    if max_pairs is None:
        max_pairs = max(1, nch * max(1, int(plan.set_max)))
    first = torch.empty(nch + 1, dtype=torch.int32, device="cuda")
    ps = torch.empty(max_pairs, dtype=torch.int16, device="cuda")
    pe = torch.empty(max_pairs, dtype=torch.int16, device="cuda")
    _check(lib().dfa_match_maps(d.handle, d_input.data_ptr() if n else None, n,
                                DFA_Q0 if start is None else int(start), ctypes.byref(o),
                                _stream_handle(stream), result.data_ptr(), first.data_ptr(),
                                ps.data_ptr(), pe.data_ptr(), int(max_pairs)))
    return result, first, ps, pe


def dfa_match_block(d: DFA, d_input, offset: int, length: int, start: Optional[int] = None,
                    chunk_len: int = 0, lookahead: int = 1, stream=None, max_entries: int = 0,
                    out=None, rounds: int = 0, single_step: bool = False,
                    interleave: bool = False, chunk_lanes: bool = False, early_exit: bool = False):
    """dfa_match_block: the block map of bytes [offset, offset + length) of the
    device string d_input.  Returns (info int32 [4], start int16 [max_entries],
    end int16 [max_entries]) device tensors (or writes into `out`, a tuple of
    such tensors)."""
    import torch
    o = _opts(chunk_len, lookahead, early_exit, rounds, single_step, interleave, chunk_lanes)
    if out is None:
        if not max_entries:
            plan = dfa_plan_info_t()
            _check(lib().dfa_plan(d.handle, int(length), ctypes.byref(o), ctypes.byref(plan)))
            max_entries = max(8, int(plan.set_max))
        out = (torch.empty(4, dtype=torch.int32, device="cuda"),
               torch.empty(max_entries, dtype=torch.int16, device="cuda"),
               torch.empty(max_entries, dtype=torch.int16, device="cuda"))
    info, st, en = out
    _check(lib().dfa_match_block(d.handle, d_input.data_ptr(), int(offset), int(length),
                                 DFA_Q0 if start is None else int(start), ctypes.byref(o),
                                 _stream_handle(stream), info.data_ptr(), st.data_ptr(),
                                 en.data_ptr(), int(st.numel())))
    return info, st, en


def dfa_compose_blocks(d: DFA, infos, starts, ends, start: Optional[int] = None, stream=None,
                       result=None, block_states=None):
    """dfa_compose_blocks over G blocks: infos int32 [G, 4], starts / ends int16
    [G, max_entries] (contiguous).  Returns (result tensor, block states int32
    [G + 1])."""
    import torch
    G = int(infos.shape[0])
    assert infos.is_contiguous() and starts.is_contiguous() and ends.is_contiguous()
    assert starts.shape == ends.shape and starts.shape[0] == G
    result = _result_tensor(result)
    if block_states is None:
        block_states = torch.empty(G + 1, dtype=torch.int32, device="cuda")
    _check(lib().dfa_compose_blocks(d.handle, G, infos.data_ptr(), starts.data_ptr(),
                                    ends.data_ptr(), int(starts.shape[1]),
                                    DFA_Q0 if start is None else int(start), _stream_handle(stream),
                                    result.data_ptr(), block_states.data_ptr()))
    return result, block_states


def dfa_match_batch(dfas: Sequence[DFA], inputs: Sequence, stream=None, results=None):
    """Many (DFA, device string) pairs in one call; returns an int32 [count, 4] tensor."""
    import torch
    count = len(dfas)
    assert len(inputs) == count
    if results is None:
        results = torch.empty((count, 4), dtype=torch.int32, device="cuda")
    hs = (ctypes.c_void_p * max(count, 1))(*[x.handle.value for x in dfas])
    ps = (ctypes.c_void_p * max(count, 1))(*[t.data_ptr() if t.numel() else None
                                             for t in inputs])
    ls = (ctypes.c_size_t * max(count, 1))(*[int(t.numel()) for t in inputs])
    _check(lib().dfa_match_batch(hs, ps, ls, count, _stream_handle(stream), results.data_ptr()))
    return results


def dfa_timing_enable(on: bool = True, stream=None) -> None:
    _check(lib().dfa_timing_enable(_stream_handle(stream), int(bool(on))))


def dfa_timing_read(stream=None) -> Tuple[float, float, int]:
    """(summed matcher-kernel ms, summed whole-call ms, calls) since the last read."""
    m, c, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint32()
    _check(lib().dfa_timing_read(_stream_handle(stream), ctypes.byref(m), ctypes.byref(c),
                                 ctypes.byref(k)))
    return float(m.value), float(c.value), int(k.value)


def dfa_timing_read_ex(stream=None) -> Tuple[float, float, float, int]:
    """(matcher ms, whole-call ms, longest single matcher launch ms, calls),
    each summed since the last read."""
    m, c, x, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_uint32()
    _check(lib().dfa_timing_read_ex(_stream_handle(stream), ctypes.byref(m), ctypes.byref(c),
                                    ctypes.byref(x), ctypes.byref(k)))
    return float(m.value), float(c.value), float(x.value), int(k.value)


def dfa_autotune(d: DFA, d_input, stream=None):
    """Tune on a device input: (lookahead r, chunk length, ms per call, early exit,
    walk rounds (0 = one), one symbol per lookup, interleaved codes, chunk lanes)."""
    o = dfa_match_opts_t()
    ms = ctypes.c_double()
    n = int(d_input.numel())
    _check(lib().dfa_autotune(d.handle, d_input.data_ptr() if n else None, n,
                              _stream_handle(stream), ctypes.byref(o), ctypes.byref(ms)))
    return (int(o.lookahead), int(o.chunk_len), float(ms.value), bool(o.flags & MATCH_EARLY_EXIT),
            (int(o.flags) >> 8) & 0xF, bool(o.flags & MATCH_SINGLE_STEP),
            bool(o.flags & MATCH_INTERLEAVE), bool(o.flags & MATCH_CHUNK_LANES))


def dfa_batch_tune(dfas: Sequence[DFA], inputs: Sequence, stream=None
                   ) -> Tuple[int, int, float, bool]:
    """Tune a batch: (chunk length, lookahead, ms per run, early exit)."""
    count = len(dfas)
    hs = (ctypes.c_void_p * max(count, 1))(*[x.handle.value for x in dfas])
    ps = (ctypes.c_void_p * max(count, 1))(*[t.data_ptr() if t.numel() else None for t in inputs])
    ls = (ctypes.c_size_t * max(count, 1))(*[int(t.numel()) for t in inputs])
    o = dfa_match_opts_t()
    ms = ctypes.c_double()
    _check(lib().dfa_batch_tune(hs, ps, ls, count, _stream_handle(stream), ctypes.byref(o),
                                ctypes.byref(ms)))
    return int(o.chunk_len), int(o.lookahead), float(ms.value), bool(o.flags & MATCH_EARLY_EXIT)


class Batch:
    """A planned batch of (DFA, device string) pairs (dfa_batch_create)."""

    def __init__(self, dfas: Sequence[DFA], inputs: Sequence, chunk_len: int = 0,
                 lookahead: int = 1, early_exit: bool = False):
        self._dfas = list(dfas)          # keep the DFAs alive
        self._inputs = list(inputs)      # and the device strings
        count = len(self._dfas)
        assert len(self._inputs) == count
        self.count = count
        hs = (ctypes.c_void_p * max(count, 1))(*[x.handle.value for x in self._dfas])
        ps = (ctypes.c_void_p * max(count, 1))(*[t.data_ptr() if t.numel() else None
                                                 for t in self._inputs])
        ls = (ctypes.c_size_t * max(count, 1))(*[int(t.numel()) for t in self._inputs])
        o = _opts(chunk_len, lookahead, early_exit)
        h = ctypes.c_void_p()
        _check(lib().dfa_batch_create(hs, ps, ls, count, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def run(self, results, stream=None):
        _check(lib().dfa_batch_run(self._h, _stream_handle(stream), results.data_ptr()))
        return results

    def graph_launch(self, results, stream):
        _check(lib().dfa_batch_graph_launch(self._h, _stream_handle(stream), results.data_ptr()))
        return results

    def info(self) -> Tuple[int, int]:
        c, t = ctypes.c_uint64(), ctypes.c_uint32()
        _check(lib().dfa_batch_info(self._h, ctypes.byref(c), ctypes.byref(t)))
        return int(c.value), int(t.value)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().dfa_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over resident DFAs (dfa_server_*)."""

    def __init__(self, budget_bytes: int = 0, max_inflight: int = 0, streams: int = 0,
                 max_batch: int = 0, slot_bytes: int = 0, lookahead: int = 0):
        o = dfa_server_opts_t(budget_bytes, max_inflight, streams, max_batch, lookahead,
                              slot_bytes)
        h = ctypes.c_void_p()
        _check(lib().dfa_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._dfas = []
        self._live = {}          # ticket -> device tensor kept alive until done

    def register(self, d: DFA) -> int:
        i = ctypes.c_uint32()
        _check(lib().dfa_server_register(self._h, d.handle, ctypes.byref(i)))
        self._dfas.append(d)
        return int(i.value)

    def submit(self, dfa_id: int, d_input, stream=None) -> int:
        """Submit a device uint8 tensor.  Its producer is torch's current
        stream (or `stream`): the server's batch waits for the work enqueued
        on it so far before it reads the input (dfa_server_submit_after)."""
        t = ctypes.c_uint64()
        n = int(d_input.numel())
        _check(lib().dfa_server_submit_after(self._h, int(dfa_id),
                                             d_input.data_ptr() if n else None, n,
                                             _stream_handle(stream), ctypes.byref(t)))
        self._live[int(t.value)] = d_input
        return int(t.value)

    def submit_ready(self, dfa_id: int, d_input) -> int:
        """Submit an input whose contents are already complete (dfa_server_submit)."""
        t = ctypes.c_uint64()
        n = int(d_input.numel())
        _check(lib().dfa_server_submit(self._h, int(dfa_id), d_input.data_ptr() if n else None, n,
                                       ctypes.byref(t)))
        self._live[int(t.value)] = d_input
        return int(t.value)

    def poll(self, ticket: int):
        r = dfa_result_t()
        rc = lib().dfa_server_poll(self._h, int(ticket), ctypes.byref(r))
        if rc == DFA_E_NOTREADY:
            return None
        _check(rc)
        self._live.pop(int(ticket), None)
        return int(r.final_state), bool(r.accepted), int(r.flags), int(r.num_chunks)

    def wait(self, ticket: int):
        r = dfa_result_t()
        _check(lib().dfa_server_wait(self._h, int(ticket), ctypes.byref(r)))
        self._live.pop(int(ticket), None)
        return int(r.final_state), bool(r.accepted), int(r.flags), int(r.num_chunks)

    def drain(self, cap: int = 4096):
        """Finished records: list of (ticket, (final, accepted, flags, chunks),
        submit_ns, done_ns), CLOCK_MONOTONIC nanoseconds."""
        if getattr(self, "_drain_buf", None) is None or len(self._drain_buf) < cap:
            self._drain_buf = (dfa_server_done_t * cap)()
        n = ctypes.c_size_t()
        _check(lib().dfa_server_drain(self._h, self._drain_buf, cap, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            e = self._drain_buf[k]
            t = int(e.ticket)
            self._live.pop(t, None)
            r = e.result
            out.append((t, (int(r.final_state), bool(r.accepted), int(r.flags), int(r.num_chunks)),
                        int(e.submit_ns), int(e.done_ns)))
        return out

    def stats(self) -> dfa_server_stats_t:
        s = dfa_server_stats_t()
        _check(lib().dfa_server_stats(self._h, ctypes.byref(s)))
        return s

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().dfa_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def result_tuple(result) -> Tuple[int, bool, int, int]:
    r = result.detach().cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    return int(r[0]), bool(r[1]), int(r[2]), int(r[3])
