"""ctypes binding of the X-engine C ABI (``include/xeng.h``), same names.

Argument marshalling only: every step of the X-engine runs in the HIP
library.  PyTorch supplies device memory (uint8 voltage tensors, int32
visibility tensors) and streams.  There is no fallback: if ``libxeng.so``
is missing or cannot be loaded, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("XENG_LIB", os.path.join(_HERE, "libxeng.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"X-engine library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build() or paper_1904_07778_amd/build.py)")
_lib = ctypes.CDLL(LIB_PATH)

XENG_OK, XENG_EINVAL, XENG_ENOMEM, XENG_EOVERFLOW, XENG_EDEVICE, XENG_ESTATE = 0, -1, -2, -3, -4, -5
XENG_DUMP_KEEP = 1 << 0
XENG_DUMP_TO_HOST = 1 << 1
XENG_PLAN_BATCH = 1 << 0
XENG_MAX_INPUTS = 256
XENG_MAX_INTEGRATION = 16_777_215


class xeng_array_desc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_chans", ctypes.c_int32),
                ("max_time_per_call", ctypes.c_int64)]


_P = ctypes.c_void_p
_lib.xeng_plan.argtypes = [ctypes.POINTER(_P), ctypes.POINTER(xeng_array_desc), ctypes.c_int32,
                           ctypes.c_uint32, _P]
_lib.xeng_plan.restype = ctypes.c_int
_lib.xeng_correlate.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64)]
_lib.xeng_correlate.restype = ctypes.c_int
_lib.xeng_dump.argtypes = [_P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.c_uint32,
                           ctypes.POINTER(ctypes.c_int64)]
_lib.xeng_dump.restype = ctypes.c_int
_lib.xeng_destroy.argtypes = [_P]
_lib.xeng_destroy.restype = None
_lib.xeng_nbaselines.argtypes = [ctypes.c_int32]
_lib.xeng_nbaselines.restype = ctypes.c_int64
_lib.xeng_baseline_index.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.xeng_baseline_index.restype = ctypes.c_int64
_lib.xeng_strerror.argtypes = [ctypes.c_int]
_lib.xeng_strerror.restype = ctypes.c_char_p
_lib.xeng_last_error.argtypes = [_P]
_lib.xeng_last_error.restype = ctypes.c_char_p
_lib.xeng_integrated.argtypes = [_P, ctypes.c_int32]
_lib.xeng_integrated.restype = ctypes.c_int64
_lib.xeng_attach.argtypes = [_P, ctypes.POINTER(xeng_array_desc), ctypes.POINTER(ctypes.c_int32)]
_lib.xeng_attach.restype = ctypes.c_int
_lib.xeng_detach.argtypes = [_P, ctypes.c_int32]
_lib.xeng_detach.restype = ctypes.c_int
_lib.xeng_slots.argtypes = [_P]
_lib.xeng_slots.restype = ctypes.c_int32
_lib.xeng_accumulator_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.xeng_accumulator_bytes.restype = ctypes.c_int64
_lib.xeng_autotune.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_float)]
_lib.xeng_autotune.restype = ctypes.c_int
_lib.xeng_requantize.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P]
_lib.xeng_requantize.restype = ctypes.c_int
_lib.xeng_eq_update.argtypes = [_P, ctypes.c_int64, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P]
_lib.xeng_eq_update.restype = ctypes.c_int
_lib.xeng_ingest.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_int32, ctypes.c_int32, _P, _P, _P]
_lib.xeng_ingest.restype = ctypes.c_int
_lib.xeng_channelise.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]
_lib.xeng_channelise.restype = ctypes.c_int
_lib.xeng_tune_cache_save.argtypes = [ctypes.c_char_p]
_lib.xeng_tune_cache_save.restype = ctypes.c_int
_lib.xeng_tune_cache_load.argtypes = [ctypes.c_char_p]
_lib.xeng_tune_cache_load.restype = ctypes.c_int
_lib.xeng_tune_cache_clear.argtypes = []
_lib.xeng_tune_cache_clear.restype = ctypes.c_int
_lib.xeng_channelise_noalloc.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P]
_lib.xeng_channelise_noalloc.restype = ctypes.c_int
_lib.xeng_channelise_spectra.argtypes = [ctypes.c_int64, ctypes.c_int32]
_lib.xeng_channelise_spectra.restype = ctypes.c_int64
_lib.xeng_channelise_table_floats.argtypes = [ctypes.c_int32]
_lib.xeng_channelise_table_floats.restype = ctypes.c_int64


class xeng_stats_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("calls", "launches", "samples", "cmacs", "bytes_in", "dumps", "bytes_out")]


_lib.xeng_correlate_dump.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64)]
_lib.xeng_correlate_dump.restype = ctypes.c_int
_lib.xeng_stats.argtypes = [_P, ctypes.POINTER(xeng_stats_t)]
_lib.xeng_stats.restype = ctypes.c_int
_lib.xeng_load_acc.argtypes = [_P, ctypes.c_int32, _P, ctypes.c_int64]
_lib.xeng_load_acc.restype = ctypes.c_int


class XengError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        text = _lib.xeng_strerror(status).decode()
        super().__init__(f"{text} ({status})" + (f": {msg}" if msg else ""))


def _check(status: int, plan=None):
    if status != XENG_OK:
        msg = _lib.xeng_last_error(plan).decode() if plan else ""
        raise XengError(status, msg)


def _ptr(x) -> int | None:
    """Raw address of a tensor/array/int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x).__name__}")


# ----------------------------------------------------------- raw C entry points
def xeng_plan(arrays: Sequence[tuple[int, int, int]], flags: int = 0, stream=None) -> int:
    """arrays: (n_inputs, n_chans, max_time_per_call) per array; stream: torch
    stream, raw hipStream_t int, or None (plan-owned stream).  Returns the handle."""
    descs = (xeng_array_desc * len(arrays))(*[xeng_array_desc(*a) for a in arrays])
    h = _P()
    s = getattr(stream, "cuda_stream", stream)
    _check(_lib.xeng_plan(ctypes.byref(h), descs, len(arrays), flags, s))
    return h.value


def xeng_correlate(plan: int, voltages: Sequence, n_time: Sequence[int]) -> None:
    n = len(n_time)
    ptrs = (_P * n)(*[_ptr(v) for v in voltages])
    ts = (ctypes.c_int64 * n)(*n_time)
    _check(_lib.xeng_correlate(plan, ptrs, ts), plan)


def xeng_dump(plan: int, array: int, dst: Sequence, flags: int = 0) -> list[int]:
    n = len(dst)
    ptrs = (_P * n)(*[_ptr(d) for d in dst])
    nint = (ctypes.c_int64 * n)()
    _check(_lib.xeng_dump(plan, array, ptrs, flags, nint), plan)
    return list(nint)


def xeng_correlate_dump(plan: int, voltages: Sequence, n_time: Sequence[int], dst: Sequence) -> list[int]:
    n = len(n_time)
    ptrs = (_P * n)(*[_ptr(v) for v in voltages])
    ts = (ctypes.c_int64 * n)(*n_time)
    outs = (_P * n)(*[_ptr(d) for d in dst])
    nint = (ctypes.c_int64 * n)()
    _check(_lib.xeng_correlate_dump(plan, ptrs, ts, outs, nint), plan)
    return list(nint)


def xeng_destroy(plan: int) -> None:
    _lib.xeng_destroy(plan)


def xeng_attach(plan: int, n_inputs: int, n_chans: int, max_time_per_call: int) -> int:
    d = xeng_array_desc(n_inputs, n_chans, max_time_per_call)
    idx = ctypes.c_int32()
    _check(_lib.xeng_attach(plan, ctypes.byref(d), ctypes.byref(idx)), plan)
    return idx.value


def xeng_detach(plan: int, index: int) -> None:
    _check(_lib.xeng_detach(plan, index), plan)


def xeng_slots(plan: int) -> int:
    return int(_lib.xeng_slots(plan))


def xeng_accumulator_bytes(n_inputs: int, n_chans: int) -> int:
    return int(_lib.xeng_accumulator_bytes(n_inputs, n_chans))


def xeng_autotune(plan: int, voltages: Sequence, n_time: Sequence[int], reps: int = 3) -> float:
    n = len(n_time)
    ptrs = (_P * n)(*[_ptr(v) for v in voltages])
    ts = (ctypes.c_int64 * n)(*n_time)
    best = ctypes.c_float()
    _check(_lib.xeng_autotune(plan, ptrs, ts, reps, ctypes.byref(best)), plan)
    return best.value


def xeng_tune_cache_save(path: str) -> None:
    _check(_lib.xeng_tune_cache_save(os.fsencode(path)))


def xeng_tune_cache_load(path: str) -> None:
    _check(_lib.xeng_tune_cache_load(os.fsencode(path)))


def xeng_tune_cache_clear() -> None:
    _check(_lib.xeng_tune_cache_clear())


def xeng_nbaselines(n: int) -> int:
    return int(_lib.xeng_nbaselines(n))


def xeng_baseline_index(i: int, j: int) -> int:
    return int(_lib.xeng_baseline_index(i, j))


def xeng_strerror(status: int) -> str:
    return _lib.xeng_strerror(status).decode()


def xeng_last_error(plan: int) -> str:
    return _lib.xeng_last_error(plan).decode()


def xeng_integrated(plan: int, array: int) -> int:
    return int(_lib.xeng_integrated(plan, array))


def xeng_stats(plan: int) -> dict:
    st = xeng_stats_t()
    _check(_lib.xeng_stats(plan, ctypes.byref(st)), plan)
    return {k: getattr(st, k) for k, _ in xeng_stats_t._fields_}


def xeng_load_acc(plan: int, array: int, src, n_integrated: int) -> None:
    _check(_lib.xeng_load_acc(plan, array, _ptr(src), n_integrated), plan)


def xeng_requantize(words, gains, out, n_time: int, n_chans: int, n_inputs: int, stream=None) -> None:
    s = getattr(stream, "cuda_stream", stream)
    _check(_lib.xeng_requantize(_ptr(words), _ptr(gains), _ptr(out), n_time, n_chans, n_inputs, s))


def requantize(words, gains, out=None, stream=None):
    """Equaliser / 4-bit requantiser (F stage): PFB words int64 (or uint64)
    [T, F, N] and gains int32 (or uint32) [F, N], CUDA tensors, -> packed
    uint8 [T, F, N], the X-engine's input.  Runs on `stream` (default: the
    current stream)."""
    import torch
    if words.dim() != 3 or gains.shape != words.shape[1:]:
        raise ValueError(f"words [T, F, N] and gains [F, N] expected, got {tuple(words.shape)} and {tuple(gains.shape)}")
    if words.element_size() != 8 or gains.element_size() != 4 or not (words.is_cuda and gains.is_cuda):
        raise ValueError("words must be 8-byte and gains 4-byte integer CUDA tensors")
    if not (words.is_contiguous() and gains.is_contiguous()):
        raise ValueError("words and gains must be contiguous")
    T, F, N = words.shape
    if out is None:
        out = torch.empty((T, F, N), dtype=torch.uint8, device=words.device)
    elif out.shape != words.shape or out.dtype != torch.uint8 or not out.is_contiguous():
        raise ValueError("out must be a contiguous uint8 tensor shaped like words")
    stream = stream if stream is not None else torch.cuda.current_stream()
    xeng_requantize(words, gains, out, T, F, N, stream)
    return out


def xeng_eq_update(vis, n_integrated: int, gains_in, gains_out, n_chans: int, n_inputs: int,
                   target_rms_x16: int, stream=None) -> None:
    s = getattr(stream, "cuda_stream", stream)
    _check(_lib.xeng_eq_update(_ptr(vis), n_integrated, _ptr(gains_in), _ptr(gains_out), n_chans, n_inputs,
                               target_rms_x16, s))


def eq_update(vis, n_integrated: int, gains, target_rms: float = 2.5, out=None, stream=None):
    """New equaliser gains (int32 [F, N] CUDA tensor, fix_18_7) from a dump
    of the requantised data (int32 [F, nbl, 2] CUDA tensor), so that the
    4-bit RMS comes to target_rms (a multiple of 1/16)."""
    import torch
    F, N = gains.shape
    if vis.dim() != 3 or vis.shape[0] != F or vis.shape[1] != N * (N + 1) // 2 or vis.dtype != torch.int32:
        raise ValueError("vis must be an int32 [F, N(N+1)/2, 2] dump matching gains [F, N]")
    if gains.element_size() != 4 or not (vis.is_cuda and gains.is_cuda and vis.is_contiguous() and gains.is_contiguous()):
        raise ValueError("gains must be a contiguous 4-byte CUDA tensor")
    tx = int(round(target_rms * 16))
    out = torch.empty_like(gains) if out is None else out
    stream = stream if stream is not None else torch.cuda.current_stream()
    xeng_eq_update(vis, n_integrated, gains, out, F, N, tx, stream)
    return out


def xeng_ingest(packets, n_packets: int, packet_stride: int, mcnt0: int, n_blocks: int, n_boards: int,
                n_chans: int, xid: int, index, out, stream=None) -> None:
    s = getattr(stream, "cuda_stream", stream)
    _check(_lib.xeng_ingest(_ptr(packets), n_packets, packet_stride, mcnt0, n_blocks, n_boards, n_chans, xid,
                            _ptr(index), _ptr(out), s))


def ingest(packets, mcnt0: int, n_blocks: int, n_boards: int, n_chans: int, xid: int, out=None, stream=None):
    """Assemble an integration block from packets (uint8 CUDA tensor
    [n_packets, stride]); returns (uint8 [8 n_blocks, n_chans, 32 n_boards],
    int32 index [n_blocks, n_boards] with -1 for lost packets)."""
    import torch
    if packets.dim() != 2 or packets.dtype != torch.uint8 or not packets.is_cuda or not packets.is_contiguous():
        raise ValueError("packets must be a contiguous uint8 CUDA tensor [n_packets, stride]")
    shape = (8 * n_blocks, n_chans, 32 * n_boards)
    out = torch.empty(shape, dtype=torch.uint8, device=packets.device) if out is None else out
    if tuple(out.shape) != shape or out.dtype != torch.uint8 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous uint8 tensor {shape}")
    index = torch.empty((n_blocks, n_boards), dtype=torch.int32, device=packets.device)
    stream = stream if stream is not None else torch.cuda.current_stream()
    xeng_ingest(packets if packets.shape[0] else None, packets.shape[0], packets.shape[1], mcnt0, n_blocks,
                n_boards, n_chans, xid, index, out, stream)
    return out, index


def xeng_channelise(adc, n_samples: int, n_inputs: int, n_chans: int, out, tables, stream=None) -> None:
    s = getattr(stream, "cuda_stream", stream)
    _check(_lib.xeng_channelise(_ptr(adc), n_samples, n_inputs, n_chans, _ptr(out), _ptr(tables), s))


def xeng_channelise_noalloc(adc, n_samples: int, n_inputs: int, n_chans: int, out, stream=None) -> None:
    s = getattr(stream, "cuda_stream", stream)
    _check(_lib.xeng_channelise_noalloc(_ptr(adc), n_samples, n_inputs, n_chans, _ptr(out), s))


def channelise(adc, n_chans: int, out=None, tables=None, stream=None):
    """F-stage channeliser: int8 CUDA tensor [N, n_samples] of ADC samples ->
    complex64 spectra [S, F, N] (time, channel, input)."""
    import torch
    if adc.dim() != 2 or adc.dtype != torch.int8 or not adc.is_cuda or not adc.is_contiguous():
        raise ValueError("adc must be a contiguous int8 CUDA tensor [n_inputs, n_samples]")
    N, S_in = adc.shape
    S = int(_lib.xeng_channelise_spectra(S_in, n_chans))
    if S < 0:
        raise ValueError("bad sizes")
    if out is None:
        out = torch.empty((S, n_chans, N), dtype=torch.complex64, device=adc.device)
    if tables is None:
        tables = torch.empty(int(_lib.xeng_channelise_table_floats(n_chans)), dtype=torch.float32,
                             device=adc.device)
    stream = stream if stream is not None else torch.cuda.current_stream()
    xeng_channelise(adc, S_in, N, n_chans, out, tables, stream)
    return out


# ------------------------------------------------------------ tensor wrapper
@dataclass
class ArraySpec:
    n_inputs: int
    n_chans: int
    max_time_per_call: int

    @property
    def nbl(self) -> int:
        return self.n_inputs * (self.n_inputs + 1) // 2


class Plan:
    """Owns one C plan; checks tensor shapes/dtypes before handing pointers over.

    Array slots are indexed as in the C ABI; ``specs[k]`` is None for a free
    slot of a batched plan (after ``detach``)."""

    def __init__(self, arrays: Sequence[tuple[int, int, int]], stream=None, batch: bool = False):
        """stream: a torch.cuda.Stream the engine runs on; by default a new one.
        batch: force the batched form (persistent graph launch) even for one or
        zero arrays; it is implied by more than one array.
        correlate() orders the engine after the caller's current stream, and
        dump() orders the caller's current stream after the engine; a caller
        that runs on the engine's stream (``with torch.cuda.stream(plan.stream)``)
        gets stream order with no waits between streams."""
        import torch
        self.specs: list[ArraySpec | None] = [ArraySpec(*a) for a in arrays]
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.batched = batch or len(self.specs) > 1
        self.handle = None
        self.handle = xeng_plan([(s.n_inputs, s.n_chans, s.max_time_per_call) for s in self.specs],
                                XENG_PLAN_BATCH if batch else 0, self.stream.cuda_stream)
        # The finalizer holds the library function itself, so a plan that is
        # still open when the interpreter shuts down is destroyed before the
        # module's globals go away (weakref.finalize runs at exit).
        self._finalizer = weakref.finalize(self, _lib.xeng_destroy, self.handle)

    def close(self):
        """Wait for the plan's work and free it (also done when the Plan is
        garbage-collected or at interpreter exit)."""
        fin = getattr(self, "_finalizer", None)
        if fin is not None and fin.alive:
            fin()
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def attach(self, n_inputs: int, n_chans: int, max_time_per_call: int) -> int:
        """Admit one more array (batched plans); returns its slot."""
        idx = xeng_attach(self.handle, n_inputs, n_chans, max_time_per_call)
        spec = ArraySpec(n_inputs, n_chans, max_time_per_call)
        if idx == len(self.specs):
            self.specs.append(spec)
        else:
            self.specs[idx] = spec
        return idx

    def detach(self, index: int) -> None:
        """Free a slot and its accumulator (waits for the engine's stream)."""
        xeng_detach(self.handle, index)
        self.specs[index] = None

    def _after_caller(self, tensors=()):
        """Order the engine's stream after the caller's current stream.  When
        the caller already runs on the engine's stream this is stream order
        and nothing is inserted: a wait across two streams costs a queue
        hand-off of tens of microseconds per call on the device."""
        import torch
        cur = torch.cuda.current_stream()
        if cur == self.stream:
            return
        self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def _caller_after(self):
        """Order the caller's current stream after the engine's stream."""
        import torch
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _marshal(self, voltages):
        import torch
        if len(voltages) != len(self.specs):
            raise ValueError("one voltage tensor (or None) per slot")
        ptrs, ts = [], []
        for v, s in zip(voltages, self.specs):
            if v is None:
                ptrs.append(None)
                ts.append(0)
                continue
            if s is None:
                raise ValueError("voltages given for a free slot")
            if v.dtype != torch.uint8 or not v.is_cuda or not v.is_contiguous():
                raise ValueError("voltages must be contiguous uint8 device tensors")
            if v.dim() != 3 or v.shape[1] != s.n_chans or v.shape[2] != s.n_inputs:
                raise ValueError(f"voltage block {tuple(v.shape)} does not match [T, {s.n_chans}, {s.n_inputs}]")
            ptrs.append(v)
            ts.append(v.shape[0])
        return ptrs, ts

    def correlate(self, voltages) -> None:
        """voltages: one uint8 CUDA tensor [T, F, N] per slot (None skips)."""
        import torch
        ptrs, ts = self._marshal(voltages)
        self._after_caller(ptrs)
        xeng_correlate(self.handle, ptrs, ts)

    def correlate_dump(self, voltages, out=None):
        """Integrate one block per slot and dump every slot given a block into
        out (device int32 [F, nbl, 2] tensors, made if None); returns (out,
        n_integrated) like dump().  Slots whose voltage entry is None keep
        integrating and get None in out."""
        import torch
        ptrs, ts = self._marshal(voltages)
        if out is None:
            out = [None if v is None else self.new_output(a) for a, v in enumerate(voltages)]
        if len(out) != len(self.specs):
            raise ValueError("one output tensor (or None) per slot")
        for a, (o, s) in enumerate(zip(out, self.specs)):
            if o is None:
                continue
            if (not o.is_cuda or o.dtype != torch.int32 or not o.is_contiguous()
                    or tuple(o.shape) != (s.n_chans, s.nbl, 2)):
                raise ValueError(f"out[{a}] must be a contiguous int32 CUDA tensor [F, nbl, 2]")
        self._after_caller(ptrs)
        n = xeng_correlate_dump(self.handle, ptrs, ts, out)
        self._caller_after()
        return out, n

    def autotune(self, voltages, reps: int = 3) -> float:
        """Pick launch shapes by timing them on these inputs (accumulators must
        be freshly dumped; they are zero afterwards).  Returns ms per call."""
        import torch
        ptrs, ts = self._marshal(voltages)
        self._after_caller()
        return xeng_autotune(self.handle, ptrs, ts, reps)

    def stats(self) -> dict:
        """Counters since the plan was made (calls, launches, samples, cmacs,
        bytes_in, dumps, bytes_out)."""
        return xeng_stats(self.handle)

    def load(self, array: int, vis, n_integrated: int) -> None:
        """Seed an array's integration from saved visibilities (int32 [F, nbl, 2],
        host or device), e.g. a KEEP dump taken earlier."""
        import torch
        s = self.specs[array]
        if tuple(vis.shape) != (s.n_chans, s.nbl, 2) or vis.dtype != torch.int32 or not vis.is_contiguous():
            raise ValueError("vis must be a contiguous int32 tensor [F, nbl, 2]")
        self.stream.wait_stream(torch.cuda.current_stream())
        xeng_load_acc(self.handle, array, vis, n_integrated)
        if vis.is_cuda:
            vis.record_stream(self.stream)
        else:
            self.stream.synchronize()   # the host buffer is read on the stream

    def new_output(self, array: int, host: bool = False):
        import torch
        s = self.specs[array]
        return torch.empty((s.n_chans, s.nbl, 2), dtype=torch.int32,
                           device="cpu" if host else "cuda", pin_memory=host)

    def dump(self, array: int = -1, out=None, keep: bool = False, to_host: bool = False):
        """Returns (list of int32 [F, nbl, 2] tensors, list of n_integrated);
        with array = -1 one entry per slot (None for a free slot)."""
        import torch
        idx = list(range(len(self.specs))) if array < 0 else [array]
        if out is None:
            out = [None if self.specs[a] is None else self.new_output(a, host=to_host) for a in idx]
        self._after_caller()   # out may come from the caller's stream
        flags = (XENG_DUMP_KEEP if keep else 0) | (XENG_DUMP_TO_HOST if to_host else 0)
        n = xeng_dump(self.handle, array, out, flags)
        if not to_host:
            self._caller_after()
        return out, n
