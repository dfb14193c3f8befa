"""Python binding of libfewha with the ABI's names: a context per configured
problem, a batch of contexts, and calls on torch device tensors.  Only
argument marshalling lives here; torch supplies device memory and streams.
"""

import ctypes
from ctypes import byref, c_double, c_int, c_long, c_void_p

import numpy as np

from . import _abi
from ._abi import FewhaError


def _check(status, ctx_handle=None, batch_handle=None):
    if status != _abi.FEWHA_OK:
        msg = ""
        if ctx_handle is not None:
            msg = _abi.fewha_last_error(ctx_handle).decode()
        elif batch_handle is not None:
            msg = _abi.fewha_batch_last_error(batch_handle).decode()
        raise FewhaError(status, msg)


def _ptr(t, n=None, dtype=None):
    """Device pointer of a contiguous CUDA float32 tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 device tensor")
    if n is not None and t.numel() < n:
        raise ValueError("tensor too small: %d < %d" % (t.numel(), n))
    return c_void_p(t.data_ptr())


def _ptr64(t, n):
    """Device pointer of a contiguous CUDA float64 tensor of at least n entries."""
    import torch
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n:
        raise ValueError("expected a contiguous float64 device tensor of %d entries" % n)
    return c_void_p(t.data_ptr())


def _tuning(tuning):
    """fewha_tuning from an int (the resident transform side) or a dict with
    keys dwt_resident, pt_rows, streams, res_split, pt_split and glob_fuse
    (missing = default)."""
    t = _abi.fewha_tuning()
    if isinstance(tuning, dict):
        t.dwt_resident = int(tuning.get("dwt_resident", 0))
        t.pt_rows = int(tuning.get("pt_rows", 0))
        t.streams = int(tuning.get("streams", 0))
        t.res_split = int(tuning.get("res_split", 0))
        t.pt_split = int(tuning.get("pt_split", 0))
        t.glob_fuse = int(tuning.get("glob_fuse", 0))
    else:
        t.dwt_resident = int(tuning)
    return t


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One configured FEWHA problem (fewha_create ... fewha_finalize).

    ``cfg`` is a configuration dict (see ``synthetic.configs``); ``device``
    is the HIP device index or -1 for a host-only context (tables only);
    ``tuning`` the launch shapes of the context's own plan: the resident
    transform side (32, 64 or 128) or a dict {"dwt_resident", "pt_rows"}
    (None = defaults)."""

    def __init__(self, cfg, device=0, tuning=None):
        self.cfg = cfg
        self.tuning = tuning
        h = c_void_p()
        _check(_abi.fewha_create(byref(h), int(device)))
        self.h = h
        self.device = device
        try:
            self._configure(cfg)
        except Exception:
            _abi.fewha_destroy(self.h)
            self.h = None
            raise
        nc, ns, nl, na, nst = c_long(), c_long(), c_long(), c_long(), c_long()
        _check(_abi.fewha_sizes(self.h, byref(nc), byref(ns), byref(nl), byref(na), byref(nst)), self.h)
        self.n_coeff, self.n_slopes, self.n_layer_pts = nc.value, ns.value, nl.value
        self.n_act, self.n_state = na.value, nst.value

    def _configure(self, cfg):
        _check(_abi.fewha_set_pupil(self.h, cfg["D"], cfg["obstruction"]), self.h)
        ws = (_abi.fewha_wfs_desc * len(cfg["wfs"]))()
        self._masks = []
        for k, w in enumerate(cfg["wfs"]):
            d = ws[k]
            d.kind = _abi.FEWHA_LGS if w["kind"] == "lgs" else _abi.FEWHA_NGS
            d.n_subap = w["n_subap"]
            d.theta_x, d.theta_y = w["theta"]
            d.H = w["H"] if w["H"] is not None else 0.0
            d.sigma = w["sigma"]
            d.launch_x, d.launch_y = w.get("launch", (0.0, 0.0))
            d.tt_removal = 1 if w.get("tt_removal") else 0
            if w.get("mask") is not None:
                m = np.ascontiguousarray(np.asarray(w["mask"], dtype=np.uint8))
                self._masks.append(m)
                d.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
        _check(_abi.fewha_set_wfs(self.h, len(cfg["wfs"]), ws), self.h)
        if any(w.get("photons") is not None for w in cfg["wfs"]):
            if not all(w.get("photons") is not None for w in cfg["wfs"]):
                raise ValueError("photon counts must be given for every sensor or none")
            ph = (c_double * len(cfg["wfs"]))(*[float(w["photons"]) for w in cfg["wfs"]])
            _check(_abi.fewha_set_photons(self.h, len(cfg["wfs"]), ph), self.h)
        ls = (_abi.fewha_layer_desc * len(cfg["layers"]))()
        for k, l in enumerate(cfg["layers"]):
            ls[k].h, ls[k].n, ls[k].levels, ls[k].cn2 = l["h"], l["n"], l["levels"], l["cn2"]
        _check(_abi.fewha_set_layers(self.h, len(cfg["layers"]), ls, cfg["domain_side"]), self.h)
        pr = cfg["prior"]
        _check(_abi.fewha_set_prior(self.h, pr["alpha"], pr["r0"], pr["L0"], pr["tau"]), self.h)
        no = cfg["noise"]
        _check(_abi.fewha_set_noise(self.h, no["alpha_eta"], no["na_fwhm"], no["spot_fwhm"]), self.h)
        _check(_abi.fewha_set_control(self.h, cfg.get("gain", 1.0)), self.h)
        loop = cfg.get("loop", "open")
        if loop not in ("open", "closed"):
            raise ValueError("loop must be 'open' or 'closed'")
        _check(_abi.fewha_set_loop(self.h, 1 if loop == "closed" else 0), self.h)
        _check(_abi.fewha_set_augmentation(self.h, int(cfg.get("augment", 0))), self.h)
        if self.tuning is not None:
            _check(_abi.fewha_set_tuning(self.h, byref(_tuning(self.tuning))), self.h)
        if cfg.get("dms") and cfg.get("fit"):
            dms = (_abi.fewha_dm_desc * len(cfg["dms"]))()
            for k, dm in enumerate(cfg["dms"]):
                dms[k].h, dms[k].n_act, dms[k].pitch = dm["h"], dm["n_act"], dm["pitch"]
            fit = cfg["fit"]
            dirs = (c_double * (2 * len(fit["directions"])))(*[v for d in fit["directions"] for v in d])
            n_fit = fit.get("n_subap", cfg["wfs"][0]["n_subap"])
            _check(_abi.fewha_set_fitting(self.h, len(cfg["dms"]), dms, len(fit["directions"]), dirs, n_fit,
                                          fit["iters"], fit["eps_rel"]), self.h)
        _check(_abi.fewha_finalize(self.h), self.h)

    def close(self, _destroy=_abi.fewha_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- tables ----
    def get_table(self, which):
        n = {_abi.FEWHA_TABLE_FILTER: 6, _abi.FEWHA_TABLE_PRIOR: self.n_coeff,
             _abi.FEWHA_TABLE_PRECOND: self.n_coeff,
             _abi.FEWHA_TABLE_MASK: sum(w["n_subap"] ** 2 for w in self.cfg["wfs"])}[which]
        out = np.zeros(n)
        _check(_abi.fewha_get_table(self.h, which, out.ctypes.data_as(ctypes.POINTER(c_double)), n), self.h)
        return out

    # ---- compute ----
    def _new(self, n):
        import torch
        return torch.empty(n, dtype=torch.float32, device="cuda:%d" % self.device)

    def _sync_stream(self):
        _check(_abi.fewha_set_stream(self.h, _stream()), self.h)

    def fewha_apply_A(self, layers, slopes=None):
        slopes = self._new(self.n_slopes) if slopes is None else slopes
        self._sync_stream()
        _check(_abi.fewha_apply_A(self.h, _ptr(layers, self.n_coeff), _ptr(slopes, self.n_slopes)), self.h)
        return slopes

    def fewha_apply_AT(self, slopes, layers=None):
        layers = self._new(self.n_coeff) if layers is None else layers
        self._sync_stream()
        _check(_abi.fewha_apply_AT(self.h, _ptr(slopes, self.n_slopes), _ptr(layers, self.n_coeff)), self.h)
        return layers

    def fewha_apply_M(self, c, out=None):
        out = self._new(self.n_coeff) if out is None else out
        self._sync_stream()
        _check(_abi.fewha_apply_M(self.h, _ptr(c, self.n_coeff), _ptr(out, self.n_coeff)), self.h)
        return out

    def fewha_rhs(self, slopes, out=None):
        out = self._new(self.n_coeff) if out is None else out
        self._sync_stream()
        _check(_abi.fewha_rhs(self.h, _ptr(slopes, self.n_slopes), _ptr(out, self.n_coeff)), self.h)
        return out

    def fewha_reconstruct(self, slopes, state, layers_out=None, dm_out=None, iters=None):
        iters = self.cfg["iters"] if iters is None else iters
        self._sync_stream()
        _check(_abi.fewha_reconstruct(self.h, _ptr(slopes, self.n_slopes), _ptr(state, self.n_state),
                                      _ptr(layers_out, self.n_coeff), _ptr(dm_out, self.n_act), int(iters)),
               self.h)

    def fewha_set_solve_coarse(self, side):
        """Coarse-level correction of the converged solves (0: Jacobi only)."""
        _check(_abi.fewha_set_solve_coarse(self.h, int(side)), self.h)

    def fewha_set_refresh(self, every):
        """Restart from the true residual every `every` frames (0 = never)."""
        _check(_abi.fewha_set_refresh(self.h, int(every)), self.h)

    def fewha_set_frame_count(self, frames):
        _check(_abi.fewha_set_frame_count(self.h, int(frames)), self.h)

    def fewha_reconstruct_streamed(self, host_slopes, state, layers_out=None, dm_out=None, iters=None, chunks=1):
        """fewha_reconstruct from slopes in a host float32 tensor (pinned for
        asynchronous copies), taken in by `chunks` sensor groups as they
        arrive.  The host tensor must stay unchanged until the stream's work
        is done."""
        import torch
        if host_slopes.is_cuda or host_slopes.dtype != torch.float32 or not host_slopes.is_contiguous() \
                or host_slopes.numel() < self.n_slopes:
            raise ValueError("expected a contiguous float32 host tensor of n_slopes entries")
        iters = self.cfg["iters"] if iters is None else iters
        self._sync_stream()
        _check(_abi.fewha_reconstruct_streamed(self.h, c_void_p(host_slopes.data_ptr()), _ptr(state, self.n_state),
                                               _ptr(layers_out, self.n_coeff), _ptr(dm_out, self.n_act),
                                               int(iters), int(chunks)), self.h)

    def fewha_reconstruct_noalloc(self, slopes, state, layers_out=None, dm_out=None, iters=None):
        """fewha_reconstruct with the work buffers in the library's static
        device scratch (no allocation in the call)."""
        iters = self.cfg["iters"] if iters is None else iters
        self._sync_stream()
        _check(_abi.fewha_reconstruct_noalloc(self.h, _ptr(slopes, self.n_slopes), _ptr(state, self.n_state),
                                              _ptr(layers_out, self.n_coeff), _ptr(dm_out, self.n_act),
                                              int(iters)), self.h)

    def fewha_solve(self, rhs, x=None, max_iters=1 << 20, rtol=1e-6):
        """x = M^{-1} rhs by PCG from 0 to a relative J^{-1}-norm residual
        rtol; returns (x, iterations, residual ratio)."""
        x = self._new(self.n_coeff) if x is None else x
        it, rel = c_int(), c_double()
        self._sync_stream()
        _check(_abi.fewha_solve(self.h, _ptr(rhs, self.n_coeff), _ptr(x, self.n_coeff), int(max_iters),
                                float(rtol), byref(it), byref(rel)), self.h)
        return x, it.value, rel.value

    def fewha_solve_map(self, slopes=None, g_layers=None, x=None, max_iters=1 << 20, rtol=1e-6):
        """x = M^{-1} W^{-T} (A^T C_hat^{-1} slopes + g_layers) (either term may
        be None), the right-hand side formed in double precision; returns
        (x, iterations, residual ratio)."""
        x = self._new(self.n_coeff) if x is None else x
        it, rel = c_int(), c_double()
        self._sync_stream()
        _check(_abi.fewha_solve_map(self.h, _ptr(slopes, self.n_slopes), _ptr(g_layers, self.n_coeff),
                                    _ptr(x, self.n_coeff), int(max_iters), float(rtol), byref(it), byref(rel)),
               self.h)
        return x, it.value, rel.value

    def fewha_apply_Winv(self, coef, out=None):
        out = self._new(self.n_coeff) if out is None else out
        self._sync_stream()
        _check(_abi.fewha_apply_Winv(self.h, _ptr(coef, self.n_coeff), _ptr(out, self.n_coeff)), self.h)
        return out

    def fewha_apply_WinvT(self, layers, out=None):
        out = self._new(self.n_coeff) if out is None else out
        self._sync_stream()
        _check(_abi.fewha_apply_WinvT(self.h, _ptr(layers, self.n_coeff), _ptr(out, self.n_coeff)), self.h)
        return out

    def fewha_param_grads(self, slopes, coef, lam, out=None):
        """[dL/dalpha, dL/dgamma_l (L), dL/dh_l (L)] through c* (float64 tensor)."""
        import torch
        n = 1 + 2 * len(self.cfg["layers"])
        out = torch.empty(n, dtype=torch.float64, device="cuda:%d" % self.device) if out is None else out
        self._sync_stream()
        _check(_abi.fewha_param_grads(self.h, _ptr(slopes, self.n_slopes), _ptr(coef, self.n_coeff),
                                      _ptr(lam, self.n_coeff), _ptr64(out, n)), self.h)
        return out

    # short aliases
    solve = fewha_solve
    solve_map = fewha_solve_map
    apply_Winv = fewha_apply_Winv
    apply_WinvT = fewha_apply_WinvT
    param_grads = fewha_param_grads
    apply_A = fewha_apply_A
    apply_AT = fewha_apply_AT
    apply_M = fewha_apply_M
    rhs = fewha_rhs
    reconstruct = fewha_reconstruct
    reconstruct_noalloc = fewha_reconstruct_noalloc
    reconstruct_streamed = fewha_reconstruct_streamed
    set_refresh = fewha_set_refresh
    set_solve_coarse = fewha_set_solve_coarse
    set_frame_count = fewha_set_frame_count


class Batch:
    """fewha_batch_create over finalized device contexts; ``tuning`` is the
    batch plan's launch shapes, as for Context (see ``autotune``)."""

    def __init__(self, ctxs, tuning=None):
        self.ctxs = list(ctxs)
        self.tuning = tuning
        arr = (c_void_p * len(self.ctxs))(*[c.h.value for c in self.ctxs])
        h = c_void_p()
        t = None if tuning is None else byref(_tuning(tuning))
        _check(_abi.fewha_batch_create_tuned(byref(h), arr, len(self.ctxs), t))
        self.h = h

    def close(self, _destroy=_abi.fewha_batch_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def fewha_batch_reconstruct(self, slopes, states, layers_out=None, dm_out=None, iters=4, use_graph=True):
        n = len(self.ctxs)

        def arr(ts, sizes):
            if ts is None:
                return None
            return (c_void_p * n)(*[(_ptr(t, s).value if t is not None else None) for t, s in zip(ts, sizes)])

        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_reconstruct(
            self.h, arr(slopes, [c.n_slopes for c in self.ctxs]), arr(states, [c.n_state for c in self.ctxs]),
            arr(layers_out, [c.n_coeff for c in self.ctxs]), arr(dm_out, [c.n_act for c in self.ctxs]),
            int(iters), 1 if use_graph else 0), batch_handle=self.h)

    def fewha_batch_set_solve_coarse(self, side):
        _check(_abi.fewha_batch_set_solve_coarse(self.h, int(side)), batch_handle=self.h)

    def fewha_batch_set_refresh(self, every):
        _check(_abi.fewha_batch_set_refresh(self.h, int(every)), batch_handle=self.h)

    def fewha_batch_set_frame_count(self, frames):
        _check(_abi.fewha_batch_set_frame_count(self.h, int(frames)), batch_handle=self.h)

    def fewha_batch_time_stage(self, stage, reps=20):
        us, wg = c_double(), c_long()
        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_time_stage(self.h, int(stage), int(reps), byref(us), byref(wg)),
               batch_handle=self.h)
        return us.value, wg.value

    def _arr(self, ts, sizes, conv=_ptr):
        n = len(self.ctxs)
        if len(ts) != n:
            raise ValueError("expected %d tensors, got %d" % (n, len(ts)))
        return (c_void_p * n)(*[conv(t, s).value for t, s in zip(ts, sizes)])

    def _new_list(self, attr):
        return [c._new(getattr(c, attr)) for c in self.ctxs]

    def fewha_batch_solve(self, rhs, x=None, max_iters=1 << 20, rtol=1e-6):
        """fewha_solve for every problem; iterates until all meet rtol."""
        x = self._new_list("n_coeff") if x is None else x
        nc = [c.n_coeff for c in self.ctxs]
        it, rel = c_int(), c_double()
        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_solve(self.h, self._arr(rhs, nc), self._arr(x, nc), int(max_iters), float(rtol),
                                      byref(it), byref(rel)), batch_handle=self.h)
        return x, it.value, rel.value

    def fewha_batch_solve_map(self, slopes=None, g_layers=None, x=None, max_iters=1 << 20, rtol=1e-6):
        """fewha_solve_map for every problem (lists of tensors, or None)."""
        x = self._new_list("n_coeff") if x is None else x
        nc = [c.n_coeff for c in self.ctxs]
        it, rel = c_int(), c_double()
        sl = None if slopes is None else self._arr(slopes, [c.n_slopes for c in self.ctxs])
        gl = None if g_layers is None else self._arr(g_layers, nc)
        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_solve_map(self.h, sl, gl, self._arr(x, nc), int(max_iters), float(rtol),
                                          byref(it), byref(rel)), batch_handle=self.h)
        return x, it.value, rel.value

    def fewha_batch_apply_Winv(self, coef, out=None):
        out = self._new_list("n_coeff") if out is None else out
        nc = [c.n_coeff for c in self.ctxs]
        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_apply_Winv(self.h, self._arr(coef, nc), self._arr(out, nc)), batch_handle=self.h)
        return out

    def fewha_batch_apply_WinvT(self, layers, out=None):
        out = self._new_list("n_coeff") if out is None else out
        nc = [c.n_coeff for c in self.ctxs]
        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_apply_WinvT(self.h, self._arr(layers, nc), self._arr(out, nc)),
               batch_handle=self.h)
        return out

    def fewha_batch_param_grads(self, slopes, coef, lam, out=None):
        import torch
        ng = [1 + 2 * len(c.cfg["layers"]) for c in self.ctxs]
        if out is None:
            out = [torch.empty(n, dtype=torch.float64, device="cuda:%d" % c.device) for n, c in zip(ng, self.ctxs)]
        nc = [c.n_coeff for c in self.ctxs]
        _check(_abi.fewha_batch_set_stream(self.h, _stream()), batch_handle=self.h)
        _check(_abi.fewha_batch_param_grads(self.h, self._arr(slopes, [c.n_slopes for c in self.ctxs]),
                                            self._arr(coef, nc), self._arr(lam, nc),
                                            self._arr(out, ng, _ptr64)), batch_handle=self.h)
        return out

    reconstruct = fewha_batch_reconstruct
    time_stage = fewha_batch_time_stage
    set_refresh = fewha_batch_set_refresh
    set_solve_coarse = fewha_batch_set_solve_coarse
    set_frame_count = fewha_batch_set_frame_count
    solve = fewha_batch_solve
    solve_map = fewha_batch_solve_map
    apply_Winv = fewha_batch_apply_Winv
    apply_WinvT = fewha_batch_apply_WinvT
    param_grads = fewha_batch_param_grads
