"""Thin Python binding of librsfstat: the same entry points as the C ABI
(rsf_resample, rsf_fstat, rsf_fstat_topk, rsf_fstat_point,
rsf_fstat_backward), with torch tensors supplying device memory and the
current stream.  Only argument marshalling happens here; every step of the
method runs in the HIP kernels behind the C ABI.
"""
import ctypes as C

import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need_cuda(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")


def plan_desc_from_workload(w):
    """rsf_plan_desc from a paper_0912_4255_amd.synth.Workload."""
    d = L.PlanDesc()
    d.n_det = len(w.detectors)
    d.nfft_policy = w.nfft_policy
    d.kernel = w.kernel
    d.taps = w.taps
    d.storage = w.storage
    d.n = w.segment.n
    d.dt = w.segment.dt
    d.t_start = w.segment.t_start
    d.f_het = w.segment.f_het
    d.f_lo = w.f_lo
    d.f_hi = w.f_hi
    e = w.eph
    d.eph = L.Ephemeris(e.au_c, e.re_c, e.p_orb, e.p_sid, e.eps, e.lambda0, e.theta0)
    for i, det in enumerate(w.detectors):
        d.det[i] = L.Detector(det.lat, det.lon, det.gamma, det.sigma2)
    return d


class Plan:
    """An rsf_plan: FFT factorisation and constant tables for one segment
    shape, detector set and interpolation kernel."""

    def __init__(self, workload=None, desc=None):
        self.lib = L.load()
        self.desc = desc if desc is not None else plan_desc_from_workload(workload)
        self.n_det = self.desc.n_det
        self.n = self.desc.n
        self._p = C.c_void_p()
        L.check(self.lib.rsf_plan_create(C.byref(self._p), C.byref(self.desc)))
        n_fft, s_lo, n_out = C.c_int64(), C.c_int64(), C.c_int64()
        l1, l2, df = C.c_int32(), C.c_int32(), C.c_double()
        L.check(self.lib.rsf_plan_query(self._p, C.byref(n_fft), C.byref(s_lo), C.byref(n_out),
                                        C.byref(l1), C.byref(l2), C.byref(df)))
        self.n_fft, self.s_lo, self.n_out = n_fft.value, s_lo.value, n_out.value
        self.fft_l1, self.fft_l2, self.df = l1.value, l2.value, df.value
        self.spin_order = 1
        self.binary = False

    @property
    def first_pass(self):
        """rsf_plan_first_pass: RSF_ROWS_GENERAL, _GENERAL_WIDE, _FIXED or _RUNTIME."""
        k = C.c_int32()
        L.check(self.lib.rsf_plan_first_pass(self._p, C.byref(k)))
        return k.value

    def set_batching(self, fb=0, templates=0):
        """rsf_plan_set_batching: spindowns sharing a first-pass row, templates per launch."""
        L.check(self.lib.rsf_plan_set_batching(self._p, fb, templates))

    def _n_fdot(self, fdot):
        """Templates in a spindown tensor: [n_fdot] at order 1, [n_fdot, s] at order s."""
        if self.spin_order == 1:
            if fdot.dim() == 2 and fdot.shape[1] == 1:
                return fdot.shape[0]
            if fdot.dim() != 1:
                raise ValueError("fdot must be [n_fdot] at spin order 1")
            return fdot.shape[0]
        if fdot.dim() != 2 or fdot.shape[1] != self.spin_order:
            raise ValueError(f"fdot must be [n_fdot, {self.spin_order}] at spin order {self.spin_order}")
        return fdot.shape[0]

    def _n_theta(self, theta):
        """Candidates in a theta tensor [n, 3 + s] = (f, f^(1) .. f^(s), alpha,
        delta), followed by (a_p, P_b, t_asc) when the plan's sources are binary."""
        width = 3 + self.spin_order + (3 if self.binary else 0)
        if theta.dim() != 2 or theta.shape[1] != width:
            raise ValueError(f"theta must be [n, {width}] at spin order {self.spin_order}"
                             + (" with a binary orbit" if self.binary else ""))
        return theta.shape[0]

    def set_binary(self, on=True):
        """rsf_plan_set_binary: sky rows become (alpha, delta, a_p, P_b, t_asc)."""
        L.check(self.lib.rsf_plan_set_binary(self._p, 1 if on else 0))
        self.binary = bool(on)

    def _n_sky(self, sky):
        width = 5 if self.binary else 2
        if sky.dim() != 2 or sky.shape[1] != width:
            raise ValueError(f"sky must be [n_sky, {width}]")
        return sky.shape[0]

    def set_spin_order(self, order):
        """rsf_plan_set_spin_order: templates carry (f^(1) .. f^(order)); fdot
        tensors are then [n_fdot, order]."""
        L.check(self.lib.rsf_plan_set_spin_order(self._p, int(order)))
        self.spin_order = int(order)

    def batching(self, n_sky=1, n_fdot=1, mode=L.RSF_MODE_BATCHED):
        """rsf_plan_batching: effective (fb, templates per launch, skies per launch)."""
        fb, g, sk = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self.lib.rsf_plan_batching(self._p, n_sky, n_fdot, mode, C.byref(fb), C.byref(g), C.byref(sk)))
        return fb.value, g.value, sk.value

    def close(self):
        if self._p:
            self.lib.rsf_plan_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------
    def workspace_bytes(self, entry, n_sky=1, n_fdot=1, mode=L.RSF_MODE_BATCHED):
        b = C.c_size_t()
        L.check(self.lib.rsf_workspace_size(self._p, entry, n_sky, n_fdot, mode, C.byref(b)))
        return b.value

    def workspace(self, entry, n_sky=1, n_fdot=1, mode=L.RSF_MODE_BATCHED, device="cuda"):
        return torch.empty(max(1, self.workspace_bytes(entry, n_sky, n_fdot, mode)), dtype=torch.uint8,
                           device=device)

    def segment(self, xs, gaps=None):
        """rsf_segment from per-detector complex64 series and int64 [g][2] gap lists."""
        if len(xs) != self.n_det:
            raise ValueError("one series per detector is required")
        seg = L.Segment()
        keep = []
        for i, x in enumerate(xs):
            _need_cuda(x, torch.complex64, "x")
            if x.numel() != self.n:
                raise ValueError("series length does not match the plan")
            seg.x[i] = x.data_ptr()
            g = None if gaps is None else gaps[i]
            if g is not None and g.numel() > 0:
                _need_cuda(g, torch.int64, "gaps")
                seg.gaps[i] = g.data_ptr()
                seg.n_gaps[i] = g.shape[0]
                keep.append(g)
            else:
                seg.gaps[i] = None
                seg.n_gaps[i] = 0
        return seg, keep

    # -- entry points ----------------------------------------------------
    def resample(self, xs, gaps, sky, ws=None):
        """rsf_resample: per detector dict(z, a, b, tm, mask, abc, u) of [n_sky, ...] tensors."""
        _need_cuda(sky, torch.float64, "sky")
        n_sky = self._n_sky(sky)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        f16 = self.desc.storage == 1
        outs, descs = [], (L.Resampled * self.n_det)()
        for i in range(self.n_det):
            o = dict(z=torch.empty((n_sky, self.n), dtype=torch.int32 if f16 else torch.complex64, device=dev),
                     a=torch.empty((n_sky, self.n), dtype=torch.float32, device=dev),
                     b=torch.empty((n_sky, self.n), dtype=torch.float32, device=dev),
                     tm=torch.empty((n_sky, self.n), dtype=torch.float64, device=dev),
                     mask=torch.empty((n_sky, (self.n + 31) // 32), dtype=torch.int32, device=dev),
                     abc=torch.empty((n_sky, 3), dtype=torch.float64, device=dev),
                     u=torch.empty((n_sky, self.n), dtype=torch.float64, device=dev))
            descs[i] = L.Resampled(o["z"].data_ptr(), o["a"].data_ptr(), o["b"].data_ptr(),
                                   o["tm"].data_ptr(), o["mask"].data_ptr(), o["abc"].data_ptr(),
                                   o["u"].data_ptr())
            outs.append(o)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_RESAMPLE, n_sky, 1, device=dev)
        L.check(self.lib.rsf_resample(self._p, C.byref(seg), _ptr(sky), n_sky, descs, _ptr(ws),
                                      ws.numel(), _stream()))
        return outs

    def fstat(self, xs, gaps, sky, fdot, mode=L.RSF_MODE_BATCHED, out=None, ws=None):
        """rsf_fstat: 2F [n_sky * n_fdot, n_out] (float32), ascending frequency."""
        _need_cuda(sky, torch.float64, "sky")
        _need_cuda(fdot, torch.float64, "fdot")
        n_sky, n_fdot = self._n_sky(sky), self._n_fdot(fdot)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        if out is None:
            out = torch.empty((n_sky * n_fdot, self.n_out), dtype=torch.float32, device=dev)
        _need_cuda(out, torch.float32, "out")
        if out.numel() < n_sky * n_fdot * self.n_out:
            raise ValueError("output too small")
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_FSTAT, n_sky, n_fdot, mode, device=dev)
        L.check(self.lib.rsf_fstat(self._p, C.byref(seg), _ptr(sky), n_sky, _ptr(fdot), n_fdot, mode,
                                   _ptr(out), _ptr(ws), ws.numel(), _stream()))
        return out

    def topk(self, xs, gaps, sky, fdot, k=10, ws=None):
        """rsf_fstat_topk: the k best (2F, sky, fdot, bin) over all templates
        and bins; returns (values float32 [k], indices int32 [k, 3])."""
        _need_cuda(sky, torch.float64, "sky")
        _need_cuda(fdot, torch.float64, "fdot")
        n_sky, n_fdot = self._n_sky(sky), self._n_fdot(fdot)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        out = torch.empty((k, 4), dtype=torch.int32, device=dev)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_TOPK, n_sky, n_fdot, device=dev)
        L.check(self.lib.rsf_fstat_topk(self._p, C.byref(seg), _ptr(sky), n_sky, _ptr(fdot), n_fdot, k,
                                        _ptr(out), _ptr(ws), ws.numel(), _stream()))
        return out[:, 0].view(torch.float32), out[:, 1:]

    def semicoherent(self, xs, gaps, sky, fdot, S, t_ref, f_lo, df_c, ws=None):
        """rsf_fstat_semicoherent: add this segment's 2F along every template's
        track to S (float32 [n_sky * n_fdot][n_c], accumulated in place)."""
        _need_cuda(sky, torch.float64, "sky")
        _need_cuda(fdot, torch.float64, "fdot")
        _need_cuda(S, torch.float32, "S")
        n_sky, n_fdot = self._n_sky(sky), self._n_fdot(fdot)
        if S.dim() != 2 or S.shape[0] != n_sky * n_fdot:
            raise ValueError("S must be [n_sky * n_fdot][n_c]")
        seg, keep = self.segment(xs, gaps)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_SEMICOHERENT, n_sky, n_fdot, device=xs[0].device)
        L.check(self.lib.rsf_fstat_semicoherent(self._p, C.byref(seg), _ptr(sky), n_sky, _ptr(fdot), n_fdot,
                                                float(t_ref), float(f_lo), float(df_c), S.shape[1], _ptr(S),
                                                _ptr(ws), ws.numel(), _stream()))
        return S

    def point(self, xs, gaps, theta, out=None, ws=None):
        """rsf_fstat_point: 2F [n] at continuous theta [n, 3 + s] =
        (f, f^(1) .. f^(s), alpha, delta), s the spin order (1: (f, fdot, alpha,
        delta)); binary sources append (a_p, P_b, t_asc)."""
        _need_cuda(theta, torch.float64, "theta")
        n = self._n_theta(theta)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=dev)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_POINT, 1, n, device=dev)
        L.check(self.lib.rsf_fstat_point(self._p, C.byref(seg), _ptr(theta), n, _ptr(out), _ptr(ws),
                                         ws.numel(), _stream()))
        return out

    def backward(self, xs, gaps, theta, g_twoF, ws=None):
        """rsf_fstat_backward: (2F [n], g_twoF * d2F/dtheta, the width of theta)."""
        _need_cuda(theta, torch.float64, "theta")
        _need_cuda(g_twoF, torch.float32, "g_twoF")
        n = self._n_theta(theta)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        twoF = torch.empty(n, dtype=torch.float32, device=dev)
        g_theta = torch.empty((n, theta.shape[1]), dtype=torch.float64, device=dev)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_BACKWARD, 1, n, device=dev)
        L.check(self.lib.rsf_fstat_backward(self._p, C.byref(seg), _ptr(theta), n, _ptr(g_twoF), _ptr(twoF),
                                            _ptr(g_theta), _ptr(ws), ws.numel(), _stream()))
        return twoF, g_theta

    def backward_static(self, xs, gaps, theta, g_twoF, twoF=None, g_theta=None):
        """rsf_fstat_backward_static: as backward, with the library's static
        device scratch instead of a workspace (outputs may be passed in)."""
        _need_cuda(theta, torch.float64, "theta")
        _need_cuda(g_twoF, torch.float32, "g_twoF")
        n = self._n_theta(theta)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        twoF = twoF if twoF is not None else torch.empty(n, dtype=torch.float32, device=dev)
        g_theta = g_theta if g_theta is not None else torch.empty((n, theta.shape[1]), dtype=torch.float64,
                                                                  device=dev)
        _need_cuda(twoF, torch.float32, "twoF")
        _need_cuda(g_theta, torch.float64, "g_theta")
        L.check(self.lib.rsf_fstat_backward_static(self._p, C.byref(seg), _ptr(theta), n, _ptr(g_twoF), _ptr(twoF),
                                                   _ptr(g_theta), _stream()))
        return twoF, g_theta

    def graph_fstat(self, xs, gaps, sky, fdot, out=None, ws=None):
        """Capture a batched rsf_fstat call into a HIP graph; returns
        (Graph, out).  Graph.launch() replays it on the current stream."""
        _need_cuda(sky, torch.float64, "sky")
        _need_cuda(fdot, torch.float64, "fdot")
        n_sky, n_fdot = self._n_sky(sky), self._n_fdot(fdot)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        if out is None:
            out = torch.empty((n_sky * n_fdot, self.n_out), dtype=torch.float32, device=dev)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_FSTAT, n_sky, n_fdot, L.RSF_MODE_BATCHED, device=dev)
        h = C.c_void_p()
        L.check(self.lib.rsf_graph_create_fstat(C.byref(h), self._p, C.byref(seg), _ptr(sky), n_sky, _ptr(fdot),
                                                n_fdot, _ptr(out), _ptr(ws), ws.numel()))
        return Graph(self.lib, h, (self, xs, gaps, keep, sky, fdot, out, ws)), out

    def graph_topk(self, xs, gaps, sky, fdot, k=10, ws=None):
        """Capture a rsf_fstat_topk call into a HIP graph; returns (Graph, values, indices)."""
        _need_cuda(sky, torch.float64, "sky")
        _need_cuda(fdot, torch.float64, "fdot")
        n_sky, n_fdot = self._n_sky(sky), self._n_fdot(fdot)
        seg, keep = self.segment(xs, gaps)
        dev = xs[0].device
        res = torch.empty((k, 4), dtype=torch.int32, device=dev)
        if ws is None:
            ws = self.workspace(L.RSF_ENTRY_TOPK, n_sky, n_fdot, device=dev)
        h = C.c_void_p()
        L.check(self.lib.rsf_graph_create_topk(C.byref(h), self._p, C.byref(seg), _ptr(sky), n_sky, _ptr(fdot),
                                               n_fdot, k, _ptr(res), _ptr(ws), ws.numel()))
        return Graph(self.lib, h, (self, xs, gaps, keep, sky, fdot, res, ws)), res[:, 0].view(torch.float32), res[:, 1:]

    def profile(self, on=True):
        """Bracket every launch of this plan with hipEvents (instrumentation)."""
        L.check(self.lib.rsf_profile_enable(self._p, 1 if on else 0))

    def profile_read(self):
        """{kernel: (launches, total_ms)} since the last read; synchronises."""
        buf = (L.KernelTime * 8)()
        n = C.c_int()
        L.check(self.lib.rsf_profile_read(self._p, buf, 8, C.byref(n)))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(n.value, 8))}

    def flags(self, ws):
        f = C.c_uint32()
        L.check(self.lib.rsf_get_flags(self._p, _ptr(ws), C.byref(f), _stream()))
        return f.value


class Graph:
    """A captured HIP graph of one batched search (rsf_graph_*).  Holds
    references to every buffer it uses."""

    def __init__(self, lib, handle, keep):
        self.lib, self._h, self._keep = lib, handle, keep

    def launch(self):
        L.check(self.lib.rsf_graph_launch(self._h, _stream()))

    def close(self):
        if self._h:
            self.lib.rsf_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _segments_args(plans, inputs):
    """Host arrays of plan pointers and segment descriptors for a
    multi-segment call; inputs[i] = (xs, gaps) of segment i."""
    if len(plans) < 1 or len(plans) != len(inputs):
        raise ValueError("one (xs, gaps) pair per plan is required")
    n_seg = len(plans)
    parr = (C.c_void_p * n_seg)(*[p._p.value for p in plans])
    sarr = (L.Segment * n_seg)()
    keep = []
    for i, (p, (xs, gaps)) in enumerate(zip(plans, inputs)):
        seg, k = p.segment(xs, gaps)
        sarr[i] = seg
        keep.append(k)
    return parr, sarr, keep


def segments_workspace(plans, n_sky, n_fdot, device="cuda"):
    """rsf_segments_workspace_size, as a uint8 device tensor."""
    lib = L.load()
    parr = (C.c_void_p * len(plans))(*[p._p.value for p in plans])
    b = C.c_size_t()
    L.check(lib.rsf_segments_workspace_size(parr, len(plans), n_sky, n_fdot, C.byref(b)))
    return torch.empty(max(1, b.value), dtype=torch.uint8, device=device)


def _check_templates(plans, sky, fdot):
    _need_cuda(sky, torch.float64, "sky")
    _need_cuda(fdot, torch.float64, "fdot")
    return plans[0]._n_sky(sky), plans[0]._n_fdot(fdot)


def fstat_topk_segments(plans, inputs, sky, fdot, k=10, ws=None):
    """rsf_fstat_topk_segments: the k best (2F, sky, fdot, bin) of every
    segment; plans[i] and inputs[i] = (xs, gaps) describe segment i.  Returns
    (values float32 [n_seg, k], indices int32 [n_seg, k, 3])."""
    n_sky, n_fdot = _check_templates(plans, sky, fdot)
    parr, sarr, keep = _segments_args(plans, inputs)
    dev = sky.device
    res = torch.empty((len(plans), k, 4), dtype=torch.int32, device=dev)
    if ws is None:
        ws = segments_workspace(plans, n_sky, n_fdot, device=dev)
    L.check(plans[0].lib.rsf_fstat_topk_segments(parr, sarr, len(plans), _ptr(sky), n_sky, _ptr(fdot), n_fdot, k,
                                                 _ptr(res), _ptr(ws), ws.numel(), _stream()))
    return res[..., 0].view(torch.float32), res[..., 1:]


def graph_topk_segments(plans, inputs, sky, fdot, k=10, ws=None):
    """The multi-segment top-k captured into one HIP graph; returns (Graph,
    values [n_seg, k], indices [n_seg, k, 3]), refreshed by every replay."""
    n_sky, n_fdot = _check_templates(plans, sky, fdot)
    parr, sarr, keep = _segments_args(plans, inputs)
    dev = sky.device
    res = torch.empty((len(plans), k, 4), dtype=torch.int32, device=dev)
    if ws is None:
        ws = segments_workspace(plans, n_sky, n_fdot, device=dev)
    h = C.c_void_p()
    L.check(plans[0].lib.rsf_graph_create_topk_segments(C.byref(h), parr, sarr, len(plans), _ptr(sky), n_sky,
                                                        _ptr(fdot), n_fdot, k, _ptr(res), _ptr(ws), ws.numel()))
    g = Graph(plans[0].lib, h, (list(plans), inputs, keep, sky, fdot, res, ws))
    return g, res[..., 0].view(torch.float32), res[..., 1:]


class FStatFn(torch.autograd.Function):
    """2F(theta) at continuous (f, f^(1) .. f^(s), alpha, delta) with a
    hand-written adjoint: forward calls rsf_fstat_point, backward
    rsf_fstat_backward (which recomputes the resampled series).  theta:
    float64 [n, 3 + s] on the GPU, s the plan's spin order."""

    @staticmethod
    def forward(ctx, theta, plan, xs, gaps):
        theta = theta.detach().contiguous()
        ctx.save_for_backward(theta)
        ctx.plan, ctx.xs, ctx.gaps = plan, xs, gaps
        return plan.point(xs, gaps, theta)

    @staticmethod
    def backward(ctx, g):
        (theta,) = ctx.saved_tensors
        _, g_theta = ctx.plan.backward(ctx.xs, ctx.gaps, theta, g.detach().float().contiguous())
        return g_theta, None, None, None


def fstat_point(plan, xs, gaps, theta):
    """Differentiable 2F at continuous parameters (see FStatFn)."""
    return FStatFn.apply(theta, plan, xs, gaps)


def sft_desc_from_set(ss):
    """rsf_sft_desc from a paper_0912_4255_amd.synth.SftSet."""
    d = L.SftDesc()
    d.n_sft = len(ss.t_sft)
    d.sft_len = ss.sft_len
    d.dt_raw = ss.dt_raw
    d.k_lo = ss.k_lo
    d.n_bins = ss.n_bins
    d.t_start = ss.t_start
    d.f_het = ss.f_het
    d.band = ss.band
    d.n_out = ss.n_out
    d.dk = ss.dk
    d.median_window = ss.median_window
    d.band_taper = ss.band_taper
    d.edge_taper_s = ss.edge_taper_s
    return d


class SftPlan:
    """An rsf_sft_plan: chunking and per-chunk transform plans of one set of
    SFT start times (paper Sec. III.B front end)."""

    def __init__(self, sft_set=None, desc=None, t_sft=None):
        import numpy as np
        self.lib = L.load()
        self.desc = desc if desc is not None else sft_desc_from_set(sft_set)
        t = np.ascontiguousarray(t_sft if t_sft is not None else sft_set.t_sft, dtype=np.float64)
        self._t = t
        self._p = C.c_void_p()
        L.check(self.lib.rsf_sft_plan_create(C.byref(self._p), C.byref(self.desc),
                                             t.ctypes.data_as(C.POINTER(C.c_double))))
        nc, ng = C.c_int64(), C.c_int64()
        L.check(self.lib.rsf_sft_plan_query(self._p, C.byref(nc), None, 0, C.byref(ng)))
        self.n_chunks = nc.value
        g = np.zeros((max(ng.value, 1), 2), dtype=np.int64)
        L.check(self.lib.rsf_sft_plan_query(self._p, None, g.ctypes.data_as(C.POINTER(C.c_int64)), ng.value,
                                            C.byref(ng)))
        self.gaps = g[:ng.value].copy()
        b = C.c_size_t()
        L.check(self.lib.rsf_sft_workspace_size(self._p, C.byref(b)))
        self.ws_bytes = b.value

    def workspace(self, device="cuda"):
        return torch.empty(max(1, self.ws_bytes), dtype=torch.uint8, device=device)

    def heterodyne(self, sft, out=None, ws=None):
        """rsf_sft_heterodyne: complex64 [n_sft][n_bins] SFT bands -> x_h [n_out]."""
        _need_cuda(sft, torch.complex64, "sft")
        if tuple(sft.shape) != (self.desc.n_sft, self.desc.n_bins):
            raise ValueError("sft must be [n_sft][n_bins]")
        out = out if out is not None else torch.empty(self.desc.n_out, dtype=torch.complex64, device=sft.device)
        _need_cuda(out, torch.complex64, "out")
        if out.numel() != self.desc.n_out:
            raise ValueError("out must hold n_out samples")
        ws = ws if ws is not None else self.workspace(sft.device)
        L.check(self.lib.rsf_sft_heterodyne(self._p, _ptr(sft), _ptr(out), _ptr(ws), ws.numel(), _stream()))
        return out

    def profile(self, on=True):
        L.check(self.lib.rsf_sft_profile_enable(self._p, 1 if on else 0))

    def profile_read(self):
        buf = (L.KernelTime * 12)()
        n = C.c_int()
        L.check(self.lib.rsf_sft_profile_read(self._p, buf, 12, C.byref(n)))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(n.value, 12))}

    def close(self):
        if self._p:
            self.lib.rsf_sft_plan_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HetdecPlan:
    """An rsf_hetdec_plan: the heterodyned low-pass taps of the time-domain
    front end (paper Sec. III.A.1)."""

    def __init__(self, n_raw, dt_raw, f_het, D, K, beta, n_out):
        self.lib = L.load()
        self.desc = L.HetdecDesc(int(n_raw), float(dt_raw), float(f_het), int(D), int(K), float(beta), int(n_out))
        self._p = C.c_void_p()
        L.check(self.lib.rsf_hetdec_plan_create(C.byref(self._p), C.byref(self.desc)))

    def run(self, x, out=None):
        """rsf_hetdec: float32 [n_raw] -> complex64 [n_out]."""
        _need_cuda(x, torch.float32, "x")
        if x.numel() != self.desc.n_raw:
            raise ValueError("x must hold n_raw samples")
        out = out if out is not None else torch.empty(self.desc.n_out, dtype=torch.complex64, device=x.device)
        _need_cuda(out, torch.complex64, "out")
        if out.numel() != self.desc.n_out:
            raise ValueError("out must hold n_out samples")
        L.check(self.lib.rsf_hetdec(self._p, _ptr(x), _ptr(out), _stream()))
        return out

    def profile(self, on=True):
        L.check(self.lib.rsf_hetdec_profile_enable(self._p, 1 if on else 0))

    def profile_read(self):
        buf = (L.KernelTime * 4)()
        n = C.c_int()
        L.check(self.lib.rsf_hetdec_profile_read(self._p, buf, 4, C.byref(n)))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(n.value, 4))}

    def close(self):
        if self._p:
            self.lib.rsf_hetdec_plan_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
