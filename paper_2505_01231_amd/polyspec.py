"""Python front end of the HIP polyspectrum library.

PyTorch supplies device memory and the HIP stream; every step of the
estimator runs inside libpolyspec.so (see include/polyspec.h for the
definitions, layouts and error behaviour).  There is no CPU fallback: a
missing library or GPU raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

_WINDOWS = {"hann": L.PS_WIN_HANN, "hann_periodic": L.PS_WIN_HANN_PERIODIC, "acg": L.PS_WIN_ACG}
_PRECISION = {"fp32": L.PS_PREC_FP32, "bf16x3": L.PS_PREC_BF16X3, "fp16x2s": L.PS_PREC_FP16X2S}
_SCHEDULE = {"batched": L.PS_SCHED_BATCHED, "per_chunk": L.PS_SCHED_PER_CHUNK}
_DTYPES = {torch.float32: L.PS_F32, torch.float64: L.PS_F64, torch.int16: L.PS_I16,
           torch.complex64: L.PS_C64, torch.complex128: L.PS_C128}


def enumerate_combos(n_channels: int, order: int):
    """Every-orbit channel combinations of the given order (host only)."""
    lib = L.load()
    n = C.c_int32(0)
    L.check(lib.ps_enumerate_combos(n_channels, order, None, C.byref(n)), "ps_enumerate_combos")
    buf = (C.c_int8 * (n.value * order))()
    L.check(lib.ps_enumerate_combos(n_channels, order, buf, C.byref(n)), "ps_enumerate_combos")
    return [tuple(buf[i * order:(i + 1) * order]) for i in range(n.value)]


def _flat(combos, arity):
    if combos is None:
        return 0, None, None
    flat = [int(c) for cb in combos for c in cb]
    if len(flat) != arity * len(combos):
        raise ValueError(f"combinations of order {arity} need {arity} channels each")
    arr = (C.c_int8 * max(1, len(flat)))(*flat)
    return len(combos), arr, C.cast(arr, C.POINTER(C.c_int8))


@dataclass
class Spectra:
    """Outputs of one record (FP64; complex values as trailing (re, im)).
    s1 [n_channels, 2] holds S1 (the windowed mean) when order 1 was requested."""
    s2: torch.Tensor | None
    s2_err: torch.Tensor | None
    s3: torch.Tensor | None
    s3_err: torch.Tensor | None
    s4: torch.Tensor | None
    s4_err: torch.Tensor | None
    n_chunks: int
    flags: int
    s1: torch.Tensor | None = None
    s1_err: torch.Tensor | None = None

    def c_struct(self) -> L.ps_output:
        """The ps_output of these tensors (NULL for the orders not held)."""
        p = Plan._ptr
        return L.ps_output(p(self.s2), p(self.s2_err), p(self.s3), p(self.s3_err), p(self.s4), p(self.s4_err),
                           p(self.s1), p(self.s1_err))

    def complex(self, name: str) -> torch.Tensor:
        return torch.view_as_complex(getattr(self, name))


class Plan:
    """A configured estimator (ps_plan_t).  ``interlaced=True`` averages the
    spectra of the frames starting at sample 0 and of the frames starting half a
    frame later (Section 3's interlaced windows; batched schedule only).
    ``estimator="natural"`` selects the biased plug-in estimator of Section 6
    instead of the k-statistics (for comparisons); ``estimator="c3opt"``
    computes S3 by c3^(opt) (Section 4.1; least variance for zero-mean,
    Gaussian-dominated coefficients, m >= 2) and keeps the k-statistics for S2
    and S4.  ``complex_signal=True``
    takes complex64 / complex128 records and returns every spectrum on the
    signed grid of ``grid`` = 2 N_f - 1 points per axis (index k + N_f - 1).
    ``s4_shift=q`` (complex plans) computes S4 on the plane parallel to the cut,
    C4(a_{k+q}, b*_{k-q}, c_{l-q}, d*_{l+q}).  ``frame_lens`` lists further
    frame lengths records may carry (``execute(..., frame_lens=...)``); all
    records of an execute share each stage's launch, and every record's spectra
    are on its own frame length's grid (``frame_info``)."""

    def __init__(self, frame_len: int, n_freq: int = 0, m: int = 10, dt: float = 1.0,
                 orders=(2, 3, 4), n_channels: int = 1, window: str = "acg",
                 window_param: float = 0.14, precision: str = "fp32", schedule: str = "batched",
                 f_max: float = 0.0, combos2=None, combos3=None, combos4=None, interlaced: bool = False,
                 estimator: str = "kstat", complex_signal: bool = False, s4_shift: int = 0,
                 frame_lens=()):
        self._lib = L.load()
        self._handle = None
        cfg = L.ps_config()
        cfg.struct_size = C.sizeof(L.ps_config)
        cfg.orders = sum(1 << o for o in orders)
        cfg.n_channels = n_channels
        cfg.frame_len = frame_len
        cfg.n_freq = n_freq
        cfg.m = m
        cfg.f_max = f_max
        cfg.dt = dt
        cfg.window_param = window_param
        cfg.window = _WINDOWS[window]
        cfg.precision = _PRECISION[precision]
        cfg.schedule = _SCHEDULE[schedule]
        cfg.interlaced = 1 if interlaced else 0
        cfg.estimator = {"kstat": L.PS_EST_KSTAT, "natural": L.PS_EST_NATURAL, "c3opt": L.PS_EST_C3OPT}[estimator]
        cfg.complex_signal = 1 if complex_signal else 0
        cfg.s4_shift = s4_shift
        fl_set = 0
        for n in frame_lens:
            if n <= 0 or n & (n - 1):
                raise ValueError(f"frame length {n} is not a power of two")
            fl_set |= 1 << (int(n).bit_length() - 1)
        cfg.frame_len_set = fl_set
        self._keep = []
        for arity, combos in ((2, combos2), (3, combos3), (4, combos4)):
            n, arr, ptr = _flat(combos, arity)
            setattr(cfg, f"n_combos{arity}", n)
            setattr(cfg, f"combos{arity}", ptr)
            self._keep.append(arr)
        h = C.c_void_p()
        L.check(self._lib.ps_plan_create(C.byref(cfg), C.byref(h)), "ps_plan_create")
        self._handle = h
        info = L.ps_plan_info()
        L.check(self._lib.ps_plan_query(h, C.byref(info)), "ps_plan_query")
        self.frame_len = info.frame_len
        self.n_freq = info.n_freq
        self.grid = info.grid                 # points per output axis
        self.complex_signal = bool(complex_signal)
        self.n_coef = info.n_coef
        self.m = info.m
        self.f_max = info.f_max
        self.sum_g = list(info.sum_g)
        self.n_channels = n_channels
        self.interlaced = bool(interlaced)
        self.orders = tuple(orders)
        self.combos2 = [tuple(info.combos2[i * 2:(i + 1) * 2]) for i in range(info.n_combos2)]
        self.combos3 = [tuple(info.combos3[i * 3:(i + 1) * 3]) for i in range(info.n_combos3)]
        self.combos4 = [tuple(info.combos4[i * 4:(i + 1) * 4]) for i in range(info.n_combos4)]
        self.frame_lens = tuple(sorted({self.frame_len, *[int(n) for n in frame_lens]}))

    def frame_info(self, frame_len: int = 0) -> dict:
        """Grid of one of the plan's frame lengths (ps_plan_frame_info)."""
        info = L.ps_plan_info()
        L.check(self._lib.ps_plan_frame_info(self._handle, frame_len, C.byref(info)), "ps_plan_frame_info")
        return {"frame_len": info.frame_len, "n_freq": info.n_freq, "n_coef": info.n_coef, "grid": info.grid,
                "f_max": info.f_max, "sum_g": list(info.sum_g)}

    # ------------------------------------------------------------------
    def close(self):
        if self._handle is not None:
            self._lib.ps_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def record(self, x: torch.Tensor, frame_len: int = 0) -> L.ps_record:
        """ps_record for a device tensor [L] (one channel) or [C, L] (channels),
        cut into frames of `frame_len` (0: the plan's frame length)."""
        if not x.is_cuda:
            raise ValueError("input must be a device tensor")
        if x.dtype not in _DTYPES:
            raise ValueError(f"unsupported dtype {x.dtype}")
        if x.dim() == 1:
            x = x.unsqueeze(0)
        if x.dim() != 2 or x.shape[0] != self.n_channels:
            raise ValueError(f"expected [{self.n_channels}, L] samples")
        if x.stride(1) != 1:
            raise ValueError("samples must be contiguous along time")
        r = L.ps_record()
        r.d_data = x.data_ptr()
        r.n_samples = x.shape[1]
        r.channel_stride = x.stride(0) if x.shape[0] > 1 else x.shape[1]
        r.dtype = _DTYPES[x.dtype]
        r.frame_len = int(frame_len)
        return r

    def record_chunks(self, rec: L.ps_record):
        """(Np, flags) of a record at its own frame length (ps_record_chunks)."""
        n = C.c_int64()
        fl = C.c_uint32()
        L.check(self._lib.ps_record_chunks(self._handle, C.byref(rec), C.byref(n), C.byref(fl)), "ps_record_chunks")
        return n.value, fl.value

    def record_info(self, n_samples: int):
        n = C.c_int64()
        fl = C.c_uint32()
        L.check(self._lib.ps_record_info(self._handle, n_samples, C.byref(n), C.byref(fl)), "ps_record_info")
        return n.value, fl.value

    def _records(self, xs, frame_lens=None):
        fls = [0] * len(xs) if frame_lens is None else [int(n) for n in frame_lens]
        if len(fls) != len(xs):
            raise ValueError("one frame length per record")
        return (L.ps_record * len(xs))(*[self.record(x, n) for x, n in zip(xs, fls)]), fls

    def workspace_bytes(self, xs, frame_lens=None) -> int:
        recs, _ = self._records(xs, frame_lens)
        n = C.c_size_t()
        L.check(self._lib.ps_workspace_size(self._handle, recs, len(xs), C.byref(n)), "ps_workspace_size")
        return n.value

    def allocate_outputs(self, device, frame_len: int = 0) -> Spectra:
        nf = self.grid if frame_len in (0, self.frame_len) else self.frame_info(frame_len)["grid"]
        f64 = dict(dtype=torch.float64, device=device)
        n2, n3, n4 = len(self.combos2), len(self.combos3), len(self.combos4)
        return Spectra(
            s2=torch.empty((n2, nf, 2), **f64) if n2 else None,
            s2_err=torch.empty((n2, nf, 2), **f64) if n2 else None,
            s3=torch.empty((n3, nf, nf, 2), **f64) if n3 else None,
            s3_err=torch.empty((n3, nf, nf, 2), **f64) if n3 else None,
            s4=torch.empty((n4, nf, nf, 2), **f64) if n4 else None,
            s4_err=torch.empty((n4, nf, nf, 2), **f64) if n4 else None,
            n_chunks=0, flags=0,
            s1=torch.empty((self.n_channels, 2), **f64) if 1 in self.orders else None,
            s1_err=torch.empty((self.n_channels, 2), **f64) if 1 in self.orders else None)

    @staticmethod
    def _ptr(t):
        return None if t is None else t.data_ptr()

    def execute(self, xs, workspace: torch.Tensor | None = None, outputs=None, stream=None, frame_lens=None):
        """Enqueue the estimator for one tensor or a list of tensors (records),
        record i cut into frames of frame_lens[i] (0 / None: the plan's).
        Returns a list of Spectra (or one Spectra for a single tensor)."""
        single = isinstance(xs, torch.Tensor)
        if single:
            xs = [xs]
            frame_lens = None if frame_lens is None else [frame_lens] if isinstance(frame_lens, int) else frame_lens
        device = xs[0].device
        recs, fls = self._records(xs, frame_lens)
        need = C.c_size_t()
        L.check(self._lib.ps_workspace_size(self._handle, recs, len(xs), C.byref(need)), "ps_workspace_size")
        if workspace is None or workspace.numel() < need.value:
            workspace = torch.empty(need.value, dtype=torch.uint8, device=device)
        if outputs is None:
            outputs = [self.allocate_outputs(device, n) for n in fls]
        outs = (L.ps_output * len(xs))()
        for i, o in enumerate(outputs):
            n, fl = self.record_chunks(recs[i])
            o.n_chunks, o.flags = n, fl
            outs[i] = o.c_struct()
        st = torch.cuda.current_stream(device) if stream is None else stream
        L.check(self._lib.ps_execute(self._handle, recs, len(xs), workspace.data_ptr(), workspace.numel(),
                                     outs, C.c_void_p(st.cuda_stream)), "ps_execute")
        self._last_workspace = workspace
        return outputs[0] if single else outputs

    def sequential(self, x, chunk_lo: int = 0, n_chunks: int | None = None,
                   workspace: torch.Tensor | None = None, stream=None) -> Spectra:
        """Sequential spectra (ps_execute_sequential): the short-time estimate of
        each chunk [chunk_lo, chunk_lo + n_chunks) of one record, not averaged.
        The returned tensors carry a leading chunk dimension; error bars are NaN
        (one chunk has no spread)."""
        rec = self.record(x)
        if n_chunks is None:
            n_chunks = max(0, self.record_info(rec.n_samples)[0] - chunk_lo)
        need = C.c_size_t()
        L.check(self._lib.ps_sequential_workspace_size(self._handle, C.byref(rec), chunk_lo, n_chunks,
                                                       C.byref(need)), "ps_sequential_workspace_size")
        device = x.device
        if workspace is None or workspace.numel() < need.value:
            workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=device)
        nf = self.grid
        f64 = dict(dtype=torch.float64, device=device)
        n2, n3, n4 = len(self.combos2), len(self.combos3), len(self.combos4)
        n1 = self.n_channels if 1 in self.orders else 0
        shape = {"s1": (n1, 2), "s2": (n2, nf, 2), "s3": (n3, nf, nf, 2), "s4": (n4, nf, nf, 2)}
        t = {}
        for key, n in (("s1", n1), ("s2", n2), ("s3", n3), ("s4", n4)):
            for suffix in ("", "_err"):
                t[key + suffix] = torch.empty((n_chunks,) + shape[key], **f64) if n else None
        res = Spectra(n_chunks=n_chunks, flags=0, **t)
        out = res.c_struct()
        st = torch.cuda.current_stream(device) if stream is None else stream
        L.check(self._lib.ps_execute_sequential(self._handle, C.byref(rec), chunk_lo, n_chunks, workspace.data_ptr(),
                                                workspace.numel(), C.byref(out), C.c_void_p(st.cuda_stream)),
                "ps_execute_sequential")
        self._last_workspace = workspace
        return res

    def full_plane(self, spectra: Spectra, order: int, combo, stream=None):
        """The spectrum of one channel combination on the signed grid (-N_f, N_f)
        (ps_full_plane), gathered from a record's outputs.  Returns (values,
        errors): [2 N_f - 1, 2] for S2, [2 N_f - 1, 2 N_f - 1, 2] for S3 / S4,
        index k + N_f - 1."""
        ref = getattr(spectra, f"s{order}")
        if ref is None:
            raise ValueError(f"order {order} was not computed")
        e = 2 * self.n_freq - 1
        shape = (e, 2) if order == 2 else (e, e, 2)
        val = torch.empty(shape, dtype=torch.float64, device=ref.device)
        err = torch.empty_like(val)
        cb = (C.c_int8 * order)(*combo)
        out = spectra.c_struct()
        st = torch.cuda.current_stream(ref.device) if stream is None else stream
        L.check(self._lib.ps_full_plane(self._handle, order, cb, C.byref(out), val.data_ptr(), err.data_ptr(),
                                        C.c_void_p(st.cuda_stream)), "ps_full_plane")
        return val, err

    def graph(self, xs, workspace: torch.Tensor | None = None, outputs=None, frame_lens=None) -> "Graph":
        """Capture the execution over these tensors/buffers as a HIP graph
        (ps_graph_create); replay with Graph.launch()."""
        single = isinstance(xs, torch.Tensor)
        if single:
            xs = [xs]
            frame_lens = None if frame_lens is None else [frame_lens] if isinstance(frame_lens, int) else frame_lens
        device = xs[0].device
        recs, fls = self._records(xs, frame_lens)
        need = C.c_size_t()
        L.check(self._lib.ps_workspace_size(self._handle, recs, len(xs), C.byref(need)), "ps_workspace_size")
        if workspace is None or workspace.numel() < need.value:
            workspace = torch.empty(need.value, dtype=torch.uint8, device=device)
        if outputs is None:
            outputs = [self.allocate_outputs(device, n) for n in fls]
        outs = (L.ps_output * len(xs))()
        for i, o in enumerate(outputs):
            o.n_chunks, o.flags = self.record_chunks(recs[i])
            outs[i] = o.c_struct()
        h = C.c_void_p()
        L.check(self._lib.ps_graph_create(self._handle, recs, len(xs), workspace.data_ptr(), workspace.numel(),
                                          outs, C.byref(h)), "ps_graph_create")
        return Graph(self, h, list(xs), workspace, outputs[0] if single else outputs)

    @property
    def tuning(self) -> dict:
        """The launch configuration (ps_plan_get_tuning)."""
        t = L.ps_tuning()
        L.check(self._lib.ps_plan_get_tuning(self._handle, C.byref(t)), "ps_plan_get_tuning")
        return {"tile_group": t.tile_group, "s3_frame_batch": t.s3_frame_batch}

    def set_tuning(self, tile_group: int = 8, s3_frame_batch: int = 0):
        """Set the launch configuration (ps_plan_set_tuning); no execute of this
        plan may be in flight."""
        t = L.ps_tuning(tile_group, s3_frame_batch)
        L.check(self._lib.ps_plan_set_tuning(self._handle, C.byref(t)), "ps_plan_set_tuning")

    def autotune(self, xs, reps: int = 3, workspace: torch.Tensor | None = None, outputs=None, stream=None,
                 frame_lens=None) -> dict:
        """Time the candidate launch configurations on these records and keep the
        fastest (ps_plan_autotune).  Returns {"best": tuning, "candidates":
        [(tuning, ms per execute), ...]}; the outputs hold the last run."""
        single = isinstance(xs, torch.Tensor)
        if single:
            xs = [xs]
        device = xs[0].device
        recs, fls = self._records(xs, frame_lens)
        need = C.c_size_t()
        L.check(self._lib.ps_workspace_size(self._handle, recs, len(xs), C.byref(need)), "ps_workspace_size")
        if workspace is None or workspace.numel() < need.value:
            workspace = torch.empty(need.value, dtype=torch.uint8, device=device)
        if outputs is None:
            outputs = [self.allocate_outputs(device, n) for n in fls]
        outs = (L.ps_output * len(xs))()
        for i, o in enumerate(outputs):
            o.n_chunks, o.flags = self.record_chunks(recs[i])
            outs[i] = o.c_struct()
        st = torch.cuda.current_stream(device) if stream is None else stream
        rep = L.ps_tune_report()
        L.check(self._lib.ps_plan_autotune(self._handle, recs, len(xs), workspace.data_ptr(), workspace.numel(),
                                           outs, int(reps), C.c_void_p(st.cuda_stream), C.byref(rep)),
                "ps_plan_autotune")
        cands = [({"tile_group": rep.cand[i].tile_group, "s3_frame_batch": rep.cand[i].s3_frame_batch}, rep.ms[i])
                 for i in range(rep.n)]
        return {"best": cands[rep.best][0], "candidates": cands}

    STAGES = ("fft", "mean", "s2", "s3", "s4", "finalize")

    def profile(self, on: bool = True):
        """Turn per-stage HIP-event timing inside ps_execute on or off."""
        L.check(self._lib.ps_profile_enable(self._handle, int(bool(on))), "ps_profile_enable")

    def profile_read(self) -> dict:
        """{stage: (milliseconds, launches)} summed since the previous read."""
        buf = (C.c_double * 12)()
        L.check(self._lib.ps_profile_read(self._handle, buf, 12), "ps_profile_read")
        return {name: (buf[i], int(buf[6 + i])) for i, name in enumerate(self.STAGES)}

    def coefficients(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        """Stage a1 alone: complex64 [C, Np*m, n_coef] (without the dt factor)."""
        rec = self.record(x)
        n_chunks, _ = self.record_info(rec.n_samples)
        F = n_chunks * self.m
        out = torch.empty((self.n_channels, F, self.n_coef, 2), dtype=torch.float32, device=x.device)
        st = torch.cuda.current_stream(x.device) if stream is None else stream
        L.check(self._lib.ps_coefficients(self._handle, C.byref(rec), out.data_ptr(),
                                          C.c_void_p(st.cuda_stream)), "ps_coefficients")
        return torch.view_as_complex(out)


class Graph:
    """A captured execution (ps_graph_t).  Keeps its inputs, workspace and
    outputs alive; ``outputs`` are refreshed by every launch."""

    def __init__(self, plan: Plan, handle, inputs, workspace, outputs):
        self._plan = plan
        self._handle = handle
        self.inputs = inputs
        self.workspace = workspace
        self.outputs = outputs

    def launch(self, stream=None):
        dev = self.workspace.device
        st = torch.cuda.current_stream(dev) if stream is None else stream
        L.check(self._plan._lib.ps_graph_launch(self._handle, C.c_void_p(st.cuda_stream)), "ps_graph_launch")
        return self.outputs

    def close(self):
        if self._handle is not None:
            self._plan._lib.ps_graph_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Streamer:
    """Time-resolved spectra of consecutive windows of a host stream
    (ps_streamer_*): each push copies one window, or up to ``windows_per_push``
    consecutive windows, from pinned host memory into a staging slot and runs
    them as one execute; the copy of the next push overlaps the estimator on
    the current one."""

    def __init__(self, plan: Plan, window_samples: int, dtype=torch.float32, depth: int = 3,
                 windows_per_push: int = 1):
        self._plan = plan
        self.window = window_samples
        self.dtype = dtype
        self.depth = depth
        self.windows_per_push = windows_per_push
        h = C.c_void_p()
        L.check(plan._lib.ps_streamer_create_multi(plan._handle, window_samples, windows_per_push, _DTYPES[dtype],
                                                   depth, C.byref(h)), "ps_streamer_create_multi")
        self._handle = h
        self.n_chunks, self.flags = plan.record_info(window_samples)

    def push(self, host_windows: torch.Tensor, outputs, stream=None) -> int:
        """Enqueue n consecutive windows (pinned host tensor holding n * C * window
        samples, window-major) writing window w into ``outputs[w]`` (a Spectra, or
        a list of n); returns the slot to wait on."""
        if host_windows.is_cuda or not host_windows.is_pinned():
            raise ValueError("windows must be pinned host tensors")
        per = self.window * self._plan.n_channels
        if host_windows.dtype != self.dtype or host_windows.numel() % per != 0:
            raise ValueError("window shape or dtype does not match the streamer")
        if not host_windows.is_contiguous():
            raise ValueError("windows must be contiguous")
        n = host_windows.numel() // per
        outs = [outputs] if isinstance(outputs, Spectra) else list(outputs)
        if len(outs) != n or not 1 <= n <= self.windows_per_push:
            raise ValueError(f"{n} windows with {len(outs)} outputs (at most {self.windows_per_push} per push)")
        arr = (L.ps_output * n)()
        for w, o in enumerate(outs):
            o.n_chunks, o.flags = self.n_chunks, self.flags
            arr[w] = o.c_struct()
        st = torch.cuda.current_stream() if stream is None else stream
        slot = C.c_int32()
        L.check(self._plan._lib.ps_streamer_push_multi(self._handle, host_windows.data_ptr(), n, arr,
                                                       C.c_void_p(st.cuda_stream), C.byref(slot)),
                "ps_streamer_push_multi")
        return slot.value

    def wait(self, slot: int):
        L.check(self._plan._lib.ps_streamer_wait(self._handle, slot), "ps_streamer_wait")

    def close(self):
        if self._handle is not None:
            self._plan._lib.ps_streamer_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def quasi_spectra(x, ms, **plan_kw) -> dict:
    """Quasi-polyspectra for several chunk lengths m (Section 8): one plan per m
    over the same record.  For a stationary signal the spectra do not depend on
    m (within their error bars); a change with m points to non-stationarity.
    Returns {m: Spectra}."""
    out = {}
    for m in ms:
        with Plan(m=m, **plan_kw) as p:
            out[m] = p.execute(x)
    torch.cuda.synchronize(x.device)
    return out


def m_dependence(a: Spectra, b: Spectra, key: str = "s4", stream=None) -> torch.Tensor:
    """Per grid point |S_a - S_b| / sqrt(sigma_a^2 + sigma_b^2) (real and
    imaginary parts separately) between two quasi-spectra of one record
    computed with different m (ps_spectra_zscore)."""
    va, ea, vb, eb = (getattr(a, key), getattr(a, key + "_err"), getattr(b, key), getattr(b, key + "_err"))
    if va.shape != vb.shape or ea.shape != va.shape or eb.shape != vb.shape:
        raise ValueError("the two spectra differ in shape")
    ts = [t.contiguous() for t in (va, ea, vb, eb)]
    out = torch.empty_like(ts[0])
    lib = L.load()
    st = torch.cuda.current_stream(out.device) if stream is None else stream
    L.check(lib.ps_spectra_zscore(ts[0].data_ptr(), ts[1].data_ptr(), ts[2].data_ptr(), ts[3].data_ptr(),
                                  ts[0].numel() // 2, out.data_ptr(), C.c_void_p(st.cuda_stream)),
            "ps_spectra_zscore")
    return out


class Accumulator:
    """Running accumulation over one long record arriving in pieces
    (ps_stream_*): ``push`` appends samples (a device tensor [L] or [C, L]),
    every completed chunk's sums go into the FP64 state, ``end`` writes the
    spectra of everything pushed so far, and ``export_state`` /
    ``import_state`` save and restore the state (bit-exact resume)."""

    def __init__(self, plan: Plan, max_push_samples: int, dtype=torch.float32):
        self._plan = plan
        self.dtype = dtype
        self.max_push = max_push_samples
        h = C.c_void_p()
        L.check(plan._lib.ps_stream_begin(plan._handle, max_push_samples, _DTYPES[dtype], C.byref(h)),
                "ps_stream_begin")
        self._handle = h
        self._keep = []

    def push(self, x: torch.Tensor, stream=None):
        rec = self._plan.record(x)
        if x.dtype != self.dtype:
            raise ValueError("dtype differs from the accumulator's")
        st = torch.cuda.current_stream(x.device) if stream is None else stream
        L.check(self._plan._lib.ps_stream_push(self._handle, rec.d_data, rec.n_samples, rec.channel_stride,
                                               C.c_void_p(st.cuda_stream)), "ps_stream_push")
        self._keep = [x]            # the samples are read when the stream runs the push

    def counts(self) -> dict:
        n, s, c = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(self._plan._lib.ps_stream_counts(self._handle, C.byref(n), C.byref(s), C.byref(c)),
                "ps_stream_counts")
        return {"chunks": n.value, "samples": s.value, "carry": c.value}

    def end(self, outputs: Spectra | None = None, device=None, stream=None) -> Spectra:
        dev = device or torch.device("cuda", torch.cuda.current_device())
        out = outputs if outputs is not None else self._plan.allocate_outputs(dev)
        out.n_chunks = self.counts()["chunks"]
        out.flags = (L.PS_FLAG_EMPTY if out.n_chunks == 0 else 0) | (L.PS_FLAG_NO_ERRBAR if out.n_chunks == 1 else 0)
        o = out.c_struct()
        st = torch.cuda.current_stream(dev) if stream is None else stream
        L.check(self._plan._lib.ps_stream_end(self._handle, C.byref(o), C.c_void_p(st.cuda_stream)),
                "ps_stream_end")
        return out

    def export_state(self) -> bytes:
        n = C.c_size_t()
        L.check(self._plan._lib.ps_stream_export_state(self._handle, None, C.byref(n)), "ps_stream_export_state")
        buf = C.create_string_buffer(n.value)
        L.check(self._plan._lib.ps_stream_export_state(self._handle, buf, C.byref(n)), "ps_stream_export_state")
        return buf.raw[: n.value]

    def import_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        L.check(self._plan._lib.ps_stream_import_state(self._handle, buf, len(state)), "ps_stream_import_state")

    def close(self):
        if self._handle is not None:
            self._plan._lib.ps_stream_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
