"""Thin ctypes binding of libni (include/ni.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Torch tensors provide device memory and the stream; the functions
keep the C names (ni_integrate, ni_label, ni_fill, ni_irls, ...).  If the
shared library is missing, loading fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libni.so")
NI_MAX_IRLS = 256

NI_OK, NI_E_ARG, NI_E_SHAPE, NI_E_NONFINITE, NI_E_NOMEM, NI_E_DEVICE, NI_E_NOTCONV, NI_E_MODEL = range(8)
NI_ORTHO, NI_PERSP = 0, 1

EXPORTED = ["ni_params_default", "ni_create", "ni_destroy", "ni_set_stream", "ni_integrate", "ni_label",
            "ni_label_noalloc", "ni_irls_step",
            "ni_fill", "ni_irls", "ni_unet_load", "ni_status_str", "ni_last_error", "ni_abi_version",
            "ni_unet_param_count", "ni_unet_blob_size", "ni_unet_init", "ni_unet_save", "ni_unet_get_params",
            "ni_unet_set_params", "ni_unet_predict", "ni_unet_forward", "ni_unet_backward", "ni_unet_train_step"]


class ni_camera(C.Structure):
    _fields_ = [("proj", C.c_int32), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("pixel_pitch", C.c_double)]


class ni_params(C.Structure):
    _fields_ = [("theta_c_deg", C.c_double), ("connectivity", C.c_int32), ("irls_iters", C.c_int32),
                ("align_iters", C.c_int32), ("bini_k", C.c_double), ("out_L", C.c_double),
                ("out_U", C.c_double), ("outlier_mode", C.c_int32), ("delta_e_max", C.c_double),
                ("w_cut_rel", C.c_double), ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int32),
                ("q_rtol", C.c_double), ("q_max_iter", C.c_int32), ("warm_start", C.c_int32),
                ("graphs", C.c_int32), ("fill_chunk", C.c_int32), ("fill_split", C.c_int32),
                ("fill_precond", C.c_int32), ("fill_mg_maxit", C.c_int32), ("freq_merging", C.c_int32),
                ("variant", C.c_int32), ("q_rtol_refine", C.c_double)]


# layout version of the structs below (NI_ABI_VERSION in include/ni.h)
ABI_VERSION = 3


class ni_report(C.Structure):
    _fields_ = [("K", C.c_int32), ("n_valid", C.c_int32), ("n_regions", C.c_int32),
                ("n_inter_edges", C.c_int32), ("n_pairs", C.c_int32), ("irls_iters_run", C.c_int32),
                ("n_small", C.c_int32), ("n_large", C.c_int32), ("fill_iters_max", C.c_int32),
                ("fill_notconv", C.c_int32), ("fill_px_iters", C.c_int64),
                ("fill_large_px_iters", C.c_int64), ("fill_large_launches", C.c_int32),
                ("warm_fallbacks", C.c_int32), ("fill_max_relres", C.c_double),
                ("quot_iters", C.c_int32 * NI_MAX_IRLS), ("energy", C.c_double * NI_MAX_IRLS),
                ("ms_setup", C.c_float), ("ms_label", C.c_float), ("ms_segments", C.c_float),
                ("ms_assemble", C.c_float), ("ms_warm", C.c_float), ("ms_fill_small", C.c_float),
                ("ms_fill_large", C.c_float), ("ms_irls", C.c_float), ("ms_finalize", C.c_float),
                ("ms_total", C.c_float), ("ms_large_kernel", C.c_float), ("fill_chunk", C.c_int32),
                ("fill_split", C.c_int32), ("fill_mg_levels", C.c_int32), ("ms_fill_mg_build", C.c_float),
                ("fill_mg_bytes", C.c_double), ("fill_mg_fallback", C.c_int32),
                ("fill_large_px", C.c_int64), ("merges", C.c_int32), ("nodes_final", C.c_int32),
                ("quot_iters_refine", C.c_int32 * NI_MAX_IRLS)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name in ("quot_iters", "energy", "quot_iters_refine"):
                v = list(v)[: max(self.irls_iters_run, 0)]
            d[name] = v
        return d


_lib = None


def lib():
    """The loaded shared library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libni.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        P = C.POINTER
        L.ni_params_default.argtypes = [P(ni_params)]
        L.ni_create.argtypes = [P(vp), C.c_int]
        L.ni_destroy.argtypes = [vp]
        L.ni_set_stream.argtypes = [vp, vp]
        L.ni_integrate.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), P(ni_params), vp, vp, vp, i64,
                                   P(i32), P(ni_report)]
        L.ni_label.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), P(ni_params), vp, P(i32), P(ni_report)]
        L.ni_irls_step.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), P(ni_params), vp, i32, vp, vp, i32, vp,
                                   P(C.c_double), P(ni_report)]
        L.ni_label_noalloc.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), P(ni_params), vp, P(i32)]
        L.ni_fill.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), P(ni_params), vp, i32, vp, P(ni_report)]
        L.ni_irls.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), P(ni_params), vp, i32, vp, vp, vp, i64,
                              P(ni_report)]
        L.ni_unet_load.argtypes = [vp, vp, C.c_size_t]
        L.ni_unet_param_count.restype = i32
        L.ni_unet_blob_size.restype = C.c_size_t
        L.ni_unet_init.argtypes = [vp, C.c_uint64]
        L.ni_unet_save.argtypes = [vp, vp, C.c_size_t]
        L.ni_unet_get_params.argtypes = [vp, vp, i32]
        L.ni_unet_set_params.argtypes = [vp, vp, i32]
        L.ni_unet_predict.argtypes = [vp, vp, vp, i32, i32, P(ni_camera), vp]
        L.ni_unet_forward.argtypes = [vp, vp, i32, i32, i32, vp]
        L.ni_unet_backward.argtypes = [vp, vp, vp]
        L.ni_unet_train_step.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, i32, C.c_float, P(C.c_double)]
        L.ni_status_str.argtypes = [C.c_int]
        L.ni_status_str.restype = C.c_char_p
        L.ni_last_error.argtypes = [vp]
        L.ni_last_error.restype = C.c_char_p
        L.ni_abi_version.restype = C.c_int32
        for name in EXPORTED:
            if name not in ("ni_status_str", "ni_last_error", "ni_abi_version", "ni_unet_param_count",
                            "ni_unet_blob_size"):
                getattr(L, name).restype = C.c_int
        if L.ni_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.ni_abi_version()}, this binding expects "
                               f"{ABI_VERSION}: rebuild the library")
        _lib = L
    return _lib


class NIError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().ni_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def ni_params_default(**overrides) -> ni_params:
    p = ni_params()
    lib().ni_params_default(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def make_camera(cam) -> ni_camera:
    """From a dict / object with proj ('ortho'|'persp'), fx, fy, cx, cy, pixel_pitch."""
    g = (lambda k: cam[k]) if isinstance(cam, dict) else (lambda k: getattr(cam, k))
    proj = g("proj")
    return ni_camera(NI_PERSP if proj == "persp" else NI_ORTHO, float(g("fx")), float(g("fy")),
                     float(g("cx")), float(g("cy")), float(g("pixel_pitch")))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _check_inputs(normals, mask):
    import torch
    if not (normals.is_cuda and mask.is_cuda):
        raise ValueError("normals and mask must be device tensors")
    if normals.dtype != torch.float32 or normals.dim() != 3 or normals.shape[2] != 3 or not normals.is_contiguous():
        raise ValueError("normals must be contiguous float32 [H, W, 3]")
    if mask.dtype != torch.uint8 or tuple(mask.shape) != tuple(normals.shape[:2]) or not mask.is_contiguous():
        raise ValueError("mask must be contiguous uint8 [H, W]")
    if normals.device != mask.device:
        raise ValueError("normals and mask on different devices")
    return normals.shape[0], normals.shape[1]


class Context:
    """Owns an ni_ctx on one device; calls run on torch's current stream."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = lib().ni_create(C.byref(h), int(device))
        if st != NI_OK:
            raise NIError(st, "ni_create failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().ni_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        import torch
        lib().ni_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _raise(self, st):
        if st != NI_OK:
            raise NIError(st, lib().ni_last_error(self.h).decode())

    def ni_integrate(self, normals, mask, cam, params=None, cap=None, raise_notconv=True):
        import torch
        H, W = _check_inputs(normals, mask)
        p = params or ni_params_default()
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        dev = normals.device
        depth = torch.empty((H, W), dtype=torch.float32, device=dev)
        labels = torch.empty((H, W), dtype=torch.int32, device=dev)
        if cap is None:
            cap = H * W
        log_scale = torch.empty((max(int(cap), 1),), dtype=torch.float64, device=dev)
        K = C.c_int32(0)
        rep = ni_report()
        self._stream()
        st = lib().ni_integrate(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), C.byref(p), _ptr(depth),
                                _ptr(labels), _ptr(log_scale), int(cap), C.byref(K), C.byref(rep))
        if st != NI_OK and not (st == NI_E_NOTCONV and not raise_notconv):
            self._raise(st)
        return dict(depth=depth, labels=labels, log_scale=log_scale[: K.value], K=K.value,
                    report=rep.as_dict(), status=st)

    def ni_label(self, normals, mask, cam, params=None):
        import torch
        H, W = _check_inputs(normals, mask)
        p = params or ni_params_default()
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        labels = torch.empty((H, W), dtype=torch.int32, device=normals.device)
        K = C.c_int32(0)
        rep = ni_report()
        self._stream()
        self._raise(lib().ni_label(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), C.byref(p),
                                   _ptr(labels), C.byref(K), C.byref(rep)))
        return labels, K.value, rep.as_dict()

    def ni_label_noalloc(self, normals, mask, cam, labels, params=None):
        """Labels into the caller's int32 [H, W] device tensor `labels`; the
        library allocates nothing (static per-GPU scratch).  Returns K."""
        import torch
        H, W = _check_inputs(normals, mask)
        p = params or ni_params_default()
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        if labels.dtype != torch.int32 or tuple(labels.shape) != (H, W) or not labels.is_contiguous():
            raise ValueError("labels must be a contiguous int32 [H, W] tensor")
        K = C.c_int32(0)
        self._stream()
        self._raise(lib().ni_label_noalloc(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), C.byref(p),
                                           _ptr(labels), C.byref(K)))
        return K.value

    def ni_fill(self, normals, mask, cam, labels, K, params=None):
        import torch
        H, W = _check_inputs(normals, mask)
        p = params or ni_params_default()
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        labels = labels.to(device=normals.device, dtype=torch.int32).contiguous()
        z = torch.empty((H, W), dtype=torch.float32, device=normals.device)
        rep = ni_report()
        self._stream()
        self._raise(lib().ni_fill(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), C.byref(p),
                                  _ptr(labels), int(K), _ptr(z), C.byref(rep)))
        return z, rep.as_dict()

    def ni_irls_step(self, normals, mask, cam, labels, K, zfill, S_in, t, params=None):
        """One relative-scale iteration t from the scales S_in (f64 [K]);
        returns (s^(t) f64 [K] device tensor, E_t, report)."""
        import torch
        H, W = _check_inputs(normals, mask)
        p = params or ni_params_default()
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        labels = labels.to(device=normals.device, dtype=torch.int32).contiguous()
        zfill = zfill.to(device=normals.device, dtype=torch.float32).contiguous()
        S_in = S_in.to(device=normals.device, dtype=torch.float64).contiguous()
        s_out = torch.empty((max(int(K), 1),), dtype=torch.float64, device=normals.device)
        e = C.c_double(0.0)
        rep = ni_report()
        self._stream()
        self._raise(lib().ni_irls_step(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), C.byref(p),
                                       _ptr(labels), int(K), _ptr(zfill), _ptr(S_in), int(t), _ptr(s_out),
                                       C.byref(e), C.byref(rep)))
        return s_out[: int(K)], e.value, rep.as_dict()

    def ni_irls(self, normals, mask, cam, labels, K, zfill, params=None):
        import torch
        H, W = _check_inputs(normals, mask)
        p = params or ni_params_default()
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        labels = labels.to(device=normals.device, dtype=torch.int32).contiguous()
        zfill = zfill.to(device=normals.device, dtype=torch.float32).contiguous()
        depth = torch.empty((H, W), dtype=torch.float32, device=normals.device)
        log_scale = torch.empty((max(int(K), 1),), dtype=torch.float64, device=normals.device)
        rep = ni_report()
        self._stream()
        self._raise(lib().ni_irls(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), C.byref(p),
                                  _ptr(labels), int(K), _ptr(zfill), _ptr(depth), _ptr(log_scale), int(K),
                                  C.byref(rep)))
        return depth, log_scale[: int(K)], rep.as_dict()

    def ni_unet_load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._raise(lib().ni_unet_load(self.h, C.cast(buf, C.c_void_p), len(blob)))

    def ni_unet_init(self, seed: int):
        self._raise(lib().ni_unet_init(self.h, C.c_uint64(seed)))

    def ni_unet_save(self) -> bytes:
        n = lib().ni_unet_blob_size()
        buf = C.create_string_buffer(n)
        self._raise(lib().ni_unet_save(self.h, C.cast(buf, C.c_void_p), n))
        return buf.raw

    def ni_unet_get_params(self):
        import numpy as np
        n = lib().ni_unet_param_count()
        out = np.empty(n, np.float32)
        self._raise(lib().ni_unet_get_params(self.h, C.c_void_p(out.ctypes.data), n))
        return out

    def ni_unet_set_params(self, prm):
        import numpy as np
        prm = np.ascontiguousarray(prm, dtype=np.float32)
        self._stream()
        self._raise(lib().ni_unet_set_params(self.h, C.c_void_p(prm.ctypes.data), prm.size))

    def ni_unet_predict(self, normals, mask, cam):
        import torch
        H, W = _check_inputs(normals, mask)
        camc = make_camera(cam) if not isinstance(cam, ni_camera) else cam
        out = torch.empty((H, W), dtype=torch.float32, device=normals.device)
        self._stream()
        self._raise(lib().ni_unet_predict(self.h, _ptr(normals), _ptr(mask), H, W, C.byref(camc), _ptr(out)))
        return out

    def ni_unet_forward(self, feat):
        import torch
        B, H, W, c6 = feat.shape
        assert c6 == 6 and feat.dtype == torch.float32 and feat.is_contiguous()
        out = torch.empty((B, H, W), dtype=torch.float32, device=feat.device)
        self._stream()
        self._raise(lib().ni_unet_forward(self.h, _ptr(feat), B, H, W, _ptr(out)))
        return out

    def ni_unet_backward(self, dout):
        import torch
        g = torch.empty((lib().ni_unet_param_count(),), dtype=torch.float32, device=dout.device)
        self._stream()
        self._raise(lib().ni_unet_backward(self.h, _ptr(dout.contiguous()), _ptr(g)))
        return g

    def ni_unet_train_step(self, normals, mask, cams, target, labels, ncomp, lr):
        """normals [B,S,S,3] f32, mask [B,S,S] u8, cams list of camera dicts,
        target [B,S,S] f32, labels [B,S,S] i32 (unique ids across the batch)."""
        B, S = normals.shape[0], normals.shape[1]
        arr = (ni_camera * B)(*[make_camera(c) for c in cams])
        loss = C.c_double(0.0)
        self._stream()
        self._raise(lib().ni_unet_train_step(self.h, _ptr(normals), _ptr(mask), C.cast(arr, C.c_void_p),
                                             _ptr(target), _ptr(labels), int(ncomp), B, S, float(lr),
                                             C.byref(loss)))
        return loss.value
