"""ctypes binding of librsc (include/rsc.h), same call names as the C ABI.

Only argument marshalling happens here: shape/dtype/device checks, output
allocation with torch, and passing raw pointers and the current HIP stream.
Every step of the coding path runs in the library's kernels.  If the library is
not built, loading fails with an error (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librsc.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "rsc.h")

RSC_OK, RSC_E_INVALID, RSC_E_NOMEM, RSC_E_DEVICE, RSC_E_UNSUPPORTED, RSC_E_NOT_READY = 0, -1, -2, -3, -4, -5
PRECISION = {"fp32": 0, "bf16": 1, "fp16": 2}
TILE = {"auto": 0, "16": 1, "32": 2}

_lib = None


class RscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rsc status {status}: {msg}")
        self.status = status


def lib():
    """Load librsc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1806_04374_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "rsc_create": [I, I, I, P, D, I, ctypes.POINTER(ctypes.c_void_p)],
        "rsc_basis_host": [I, I, I, P, D, P, P, P, P, P],
        "rsc_create_annular": [I, I, ctypes.POINTER(ctypes.c_void_p)],
        "rsc_annular_basis_host": [I, I, P, P, P, P, P],
        "rsc_destroy": [P],
        "rsc_basis_info": [P, P, P, P],
        "rsc_get_basis": [P, P, P],
        "rsc_set_dictionary": [P, P, I, I, P],
        "rsc_encode_workspace_size": [P, I64, I, P],
        "rsc_set_fault": [P, ctypes.c_char_p],
        "rsc_set_tile": [P, I],
        "rsc_set_launch": [P, I, I],
        "rsc_get_launch": [P, P, P],
        "rsc_encode_info": [P, I, P, P],
        "rsc_autotune_encode": [P, P, I64, I, P, P, P, I, P, P, P],
        "rsc_project": [P, P, I64, P, P],
        "rsc_omp_encode": [P, P, I64, I, P, ctypes.c_size_t, P, P, P, P, P],
        "rsc_reconstruct": [P, P, P, P, I64, I, P, P],
        "rsc_synthesize": [P, P, P, P, I64, I, P, P, P],
        "rsc_sync": [P, P],
        "rsc_images_workspace_size": [I, P],
        "rsc_project_images": [P, P, P, P, P, I, I64, P, ctypes.c_size_t, P, P],
        "rsc_project_images_noalloc": [P, P, P, P, P, I, I64, P, P],
        "rsc_synthesize_images": [P, P, P, P, P, P, I64, P, P, P, I, P, P],
        "rsc_precision_stats": [P, P, I],
        "rsc_rksvd_workspace_size": [P, I64, I, P],
        "rsc_rksvd_update": [P, P, I64, I, P, P, P, P, P, ctypes.c_size_t, P, P, P, P],
        "rsc_rksvd_train": [P, P, I64, I, I, P, I, I, P, ctypes.c_size_t, P, P, P, P, P, P, P],
        "rsc_classify_workspace_size": [I64, I, P],
        "rsc_classify": [P, I, P, I64, I, P, ctypes.c_size_t, P, P, P],
        "rsc_label_histogram": [P, I64, P, I, I, P, P],
        "rsc_chi2_nearest": [P, I, P, I, I, P, P, P],
        "rsc_rotation_plan_create": [I, ctypes.c_double, I, P],
        "rsc_rotation_plan_create_steer": [P, ctypes.c_double, P],
        "rsc_rotation_plan_destroy": [P],
        "rsc_rotate_interp": [P, P, I64, P, P],
        "rsc_steer": [P, P, I64, P, ctypes.c_double, P, P],
        "rsc_synthesize_hat": [P, P, I64, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.rsc_last_error.argtypes = [P]
    L.rsc_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in include/rsc.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"\b(rsc_\w+)\s*\(", text)


def _check(status: int):
    if status != RSC_OK:
        raise RscError(status, lib().rsc_last_error(None).decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Handle:
    """Owner of an rsc_handle*; geometry and dictionary sizes are cached."""

    def __init__(self, ptr, N, S, T, prec="fp32"):
        self.ptr = ptr
        self.N, self.S, self.T = N, S, T
        self.prec = prec
        n_pix, B, cond = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().rsc_basis_info(ptr, ctypes.byref(n_pix), ctypes.byref(B), ctypes.byref(cond)))
        self.n_pix, self.B, self.cond = n_pix.value, B.value, cond.value
        self.M = self.R = None

    def close(self):
        if self.ptr:
            lib().rsc_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rsc_create(N: int, S: int, T: int, centres=None, sigma: float = 0.0, prec: str = "fp32") -> Handle:
    h = ctypes.c_void_p()
    c = None
    if centres is not None:
        c = np.ascontiguousarray(centres, dtype=np.float64)
    _check(lib().rsc_create(N, S, T, None if c is None else c.ctypes.data_as(ctypes.c_void_p),
                            float(sigma), PRECISION[prec], ctypes.byref(h)))
    return Handle(h, N, S, T, prec)


def rsc_basis_host(N: int, S: int, T: int, centres=None, sigma: float = 0.0):
    """FP64 (phi [N*N, B], pinv [B, N*N], cond) built by the library on the host."""
    B = S * (2 * T + 1)
    phi = np.zeros((N * N, B))
    pinv = np.zeros((B, N * N))
    cond = ctypes.c_double()
    c = None if centres is None else np.ascontiguousarray(centres, dtype=np.float64)
    _check(lib().rsc_basis_host(N, S, T, None if c is None else c.ctypes.data_as(ctypes.c_void_p),
                                float(sigma), phi.ctypes.data_as(ctypes.c_void_p),
                                pinv.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(cond)))
    return phi, pinv, cond.value


def rsc_annular_basis_host(N: int, lowpass: bool = False):
    """The library's FP64 annular basis built on the host: (phi [N*N, B], pinv [B, N*N],
    per-annulus cut-offs T_s, cond)."""
    B = ctypes.c_int()
    Ts = np.zeros(N // 2, dtype=np.int32)
    _check(lib().rsc_annular_basis_host(N, int(bool(lowpass)), None, None, Ts.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(B), None))
    phi = np.zeros((N * N, B.value))
    pinv = np.zeros((B.value, N * N))
    cond = ctypes.c_double()
    _check(lib().rsc_annular_basis_host(N, int(bool(lowpass)), phi.ctypes.data_as(ctypes.c_void_p),
                                        pinv.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(cond)))
    return phi, pinv, [int(t) for t in Ts], cond.value


def rsc_create_annular(N: int, lowpass: bool = False) -> Handle:
    """FP32 handle on the paper's annular basis (projection, steering, synthesis)."""
    _, _, Ts, _ = rsc_annular_basis_host(N, lowpass)
    h = ctypes.c_void_p()
    _check(lib().rsc_create_annular(N, int(bool(lowpass)), ctypes.byref(h)))
    hd = Handle(h, N, N // 2, max(Ts), "fp32")
    hd.Ts = Ts
    return hd


def rsc_get_basis(h: Handle):
    phi = np.zeros((h.N * h.N, h.B))
    pinv = np.zeros((h.B, h.N * h.N))
    _check(lib().rsc_get_basis(h.ptr, phi.ctypes.data_as(ctypes.c_void_p),
                               pinv.ctypes.data_as(ctypes.c_void_p)))
    return phi, pinv


def rsc_set_dictionary(h: Handle, d_hat, R: int, stream=None):
    """Uploads the host dictionary [M, B] on the stream (the current one by default)."""
    d = np.ascontiguousarray(d_hat, dtype=np.float32)
    if d.ndim != 2 or d.shape[1] != h.B:
        raise ValueError(f"d_hat must be [M, {h.B}]")
    _check(lib().rsc_set_dictionary(h.ptr, d.ctypes.data_as(ctypes.c_void_p), d.shape[0], R, _stream(stream)))
    h.M, h.R = d.shape[0], R


def rsc_encode_workspace_size(h: Handle, P: int, K: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().rsc_encode_workspace_size(h.ptr, int(P), int(K), ctypes.byref(n)))
    return n.value


def rsc_set_fault(h: Handle, msg: str | None = None):
    _check(lib().rsc_set_fault(h.ptr, None if msg is None else msg.encode()))


def rsc_set_tile(h: Handle, tile: str = "auto"):
    """Encoder tile shape: "auto", "16" (16x16x4 MFMA tiles) or "32" (32x32x2)."""
    _check(lib().rsc_set_tile(h.ptr, TILE[str(tile)]))


def rsc_set_launch(h: Handle, tile: str = "auto", blocks_per_cu: int = 0):
    _check(lib().rsc_set_launch(h.ptr, TILE[str(tile)], int(blocks_per_cu)))


def rsc_encode_info(h: Handle, K: int):
    """(tile actually used for K, executed MFMA flops per patch)."""
    t, f = ctypes.c_int(), ctypes.c_double()
    _check(lib().rsc_encode_info(h.ptr, K, ctypes.byref(t), ctypes.byref(f)))
    return {v: k for k, v in TILE.items()}[t.value], f.value


def rsc_get_launch(h: Handle):
    t, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().rsc_get_launch(h.ptr, ctypes.byref(t), ctypes.byref(b)))
    return {v: k for k, v in TILE.items()}[t.value], b.value


def rsc_autotune_encode(h: Handle, xhat, K: int, reps: int = 5, stream=None):
    """Times the encoder launch shapes on the sample xhat and keeps the fastest.
    Returns [(tile, blocks_per_cu, median_ms), ...]."""
    import torch
    P = xhat.shape[0]
    _dev(xhat, torch.float32, "xhat", (P, h.B))
    atom = torch.empty((P, K), dtype=torch.int32, device=xhat.device)
    angle = torch.empty_like(atom)
    coef = torch.empty((P, K), dtype=torch.float32, device=xhat.device)
    rep = np.zeros((8, 3))
    n = ctypes.c_int()
    _check(lib().rsc_autotune_encode(h.ptr, _ptr(xhat), P, K, _ptr(atom), _ptr(angle), _ptr(coef), reps,
                                     rep.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n), _stream(stream)))
    names = {v: k for k, v in TILE.items()}
    return [(names[int(r[0])], int(r[1]), float(r[2])) for r in rep[:n.value]]


def rsc_project(h: Handle, patches, xhat=None, stream=None):
    import torch
    P = patches.shape[0]
    _dev(patches, torch.float32, "patches", (P, h.N, h.N))
    if xhat is None:
        xhat = torch.empty((P, h.B), dtype=torch.float32, device=patches.device)
    _dev(xhat, torch.float32, "xhat", (P, h.B))
    _check(lib().rsc_project(h.ptr, _ptr(patches), P, _ptr(xhat), _stream(stream)))
    return xhat


def rsc_omp_encode(h: Handle, xhat, K: int, out=None, stream=None, workspace=None):
    """Returns (atom [P,K] int32, angle [P,K] int32, coef [P,K] f32, resid2 [P] f32).
    workspace: optional device uint8 tensor (rsc_encode_workspace_size bytes, which is 0)."""
    import torch
    P = xhat.shape[0]
    _dev(xhat, torch.float32, "xhat", (P, h.B))
    if out is None:
        dv = xhat.device
        out = (torch.empty((P, K), dtype=torch.int32, device=dv),
               torch.empty((P, K), dtype=torch.int32, device=dv),
               torch.empty((P, K), dtype=torch.float32, device=dv),
               torch.empty((P,), dtype=torch.float32, device=dv))
    atom, angle, coef, resid2 = out
    _dev(atom, torch.int32, "atom", (P, K))
    _dev(angle, torch.int32, "angle", (P, K))
    _dev(coef, torch.float32, "coef", (P, K))
    if resid2 is not None:
        _dev(resid2, torch.float32, "resid2", (P,))
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().rsc_omp_encode(h.ptr, _ptr(xhat), P, K, _ptr(workspace), ws_bytes, _ptr(atom), _ptr(angle),
                                _ptr(coef), _ptr(resid2), _stream(stream)))
    return atom, angle, coef, resid2


def rsc_reconstruct(h: Handle, atom, angle, coef, out=None, stream=None):
    import torch
    P, K = atom.shape
    _dev(atom, torch.int32, "atom", (P, K))
    _dev(angle, torch.int32, "angle", (P, K))
    _dev(coef, torch.float32, "coef", (P, K))
    if out is None:
        out = torch.empty((P, h.N, h.N), dtype=torch.float32, device=atom.device)
    _dev(out, torch.float32, "out", (P, h.N, h.N))
    _check(lib().rsc_reconstruct(h.ptr, _ptr(atom), _ptr(angle), _ptr(coef), P, K, _ptr(out),
                                 _stream(stream)))
    return out


def rsc_synthesize(h: Handle, atom, theta, weight, noise=None, out=None, stream=None):
    import torch
    P, J = atom.shape
    _dev(atom, torch.int32, "atom", (P, J))
    _dev(theta, torch.float32, "theta", (P, J))
    _dev(weight, torch.float32, "weight", (P, J))
    if noise is not None:
        _dev(noise, torch.float32, "noise", (P, h.N, h.N))
    if out is None:
        out = torch.empty((P, h.N, h.N), dtype=torch.float32, device=atom.device)
    _dev(out, torch.float32, "out", (P, h.N, h.N))
    _check(lib().rsc_synthesize(h.ptr, _ptr(atom), _ptr(theta), _ptr(weight), P, J, _ptr(noise),
                                _ptr(out), _stream(stream)))
    return out


class ImageBatch:
    """Device description of a batch of images packed back to back (row-major).

    Holds the device arrays img_offset (int64), H, W (int32) and the workspace that
    rsc_project_images needs, plus the host copies of the sizes.
    """

    def __init__(self, sizes, N: int, device, offsets=None):
        """sizes: [(H, W)]; offsets: element offset of each image in the pixel buffer
        (default: images packed back to back)."""
        import torch
        sizes = np.asarray(sizes, dtype=np.int64).reshape(-1, 2)
        self.n = len(sizes)
        self.H = sizes[:, 0].copy()
        self.W = sizes[:, 1].copy()
        if offsets is None:
            off = np.zeros(self.n, np.int64)
            if self.n:
                off[1:] = np.cumsum(self.H * self.W)[:-1]
        else:
            off = np.asarray(offsets, dtype=np.int64).reshape(-1)
            if off.shape[0] != self.n or (self.n and off.min() < 0):
                raise ValueError("offsets must be one non-negative offset per image")
        self.offset = off
        self.total_pixels = int((self.H * self.W).sum())
        self.min_pixels = int((off + self.H * self.W).max()) if self.n else 0
        self.patches_per_image = np.maximum(self.H - N + 1, 0) * np.maximum(self.W - N + 1, 0)
        self.P_total = int(self.patches_per_image.sum())
        self.d_offset = torch.from_numpy(off).to(device)
        self.d_H = torch.from_numpy(self.H.astype(np.int32)).to(device)
        self.d_W = torch.from_numpy(self.W.astype(np.int32)).to(device)
        nb = ctypes.c_size_t()
        _check(lib().rsc_images_workspace_size(self.n, ctypes.byref(nb)))
        self.workspace = torch.empty(max(nb.value // 8, 1), dtype=torch.int64, device=device)
        self.ws_bytes = nb.value


def rsc_images_workspace_size(n_images: int) -> int:
    nb = ctypes.c_size_t()
    _check(lib().rsc_images_workspace_size(n_images, ctypes.byref(nb)))
    return nb.value


def rsc_project_images(h: Handle, pixels, batch: "ImageBatch", xhat=None, stream=None):
    """Hat coordinates of every stride-1 window of every image: [P_total, B]."""
    import torch
    _dev(pixels, torch.float32, "pixels")
    if pixels.dim() != 1 or pixels.shape[0] < batch.min_pixels:
        raise ValueError(f"pixels must be 1-D with at least {batch.min_pixels} elements")
    if xhat is None:
        xhat = torch.empty((batch.P_total, h.B), dtype=torch.float32, device=pixels.device)
    _dev(xhat, torch.float32, "xhat", (batch.P_total, h.B))
    _check(lib().rsc_project_images(h.ptr, _ptr(pixels), _ptr(batch.d_offset), _ptr(batch.d_H),
                                    _ptr(batch.d_W), batch.n, batch.P_total, _ptr(batch.workspace),
                                    batch.ws_bytes, _ptr(xhat), _stream(stream)))
    return xhat


def rsc_project_images_noalloc(h: Handle, pixels, batch: "ImageBatch", xhat, stream=None):
    """rsc_project_images through the entry point that allocates nothing (the plan lives
    in the library's static device buffer; batch.workspace is not used).  xhat must be
    given: device [P_total, B] float32."""
    import torch
    _dev(pixels, torch.float32, "pixels")
    if pixels.dim() != 1 or pixels.shape[0] < batch.min_pixels:
        raise ValueError(f"pixels must be 1-D with at least {batch.min_pixels} elements")
    _dev(xhat, torch.float32, "xhat", (batch.P_total, h.B))
    _check(lib().rsc_project_images_noalloc(h.ptr, _ptr(pixels), _ptr(batch.d_offset), _ptr(batch.d_H),
                                            _ptr(batch.d_W), batch.n, batch.P_total, _ptr(xhat),
                                            _stream(stream)))
    return xhat


def rsc_synthesize_images(h: Handle, batch: "ImageBatch", atom, theta, amplitude, centre, image,
                          pixels, stream=None):
    """Adds stamps to pixels (device float32 [total_pixels], initialised by the caller)."""
    import torch
    n = atom.shape[0]
    _dev(atom, torch.int32, "atom", (n,))
    _dev(theta, torch.float32, "theta", (n,))
    _dev(amplitude, torch.float32, "amplitude", (n,))
    _dev(centre, torch.int32, "centre", (n, 2))
    _dev(image, torch.int32, "image", (n,))
    _dev(pixels, torch.float32, "pixels")
    if pixels.dim() != 1 or pixels.shape[0] < batch.min_pixels:
        raise ValueError(f"pixels must be 1-D with at least {batch.min_pixels} elements")
    _check(lib().rsc_synthesize_images(h.ptr, _ptr(atom), _ptr(theta), _ptr(amplitude), _ptr(centre),
                                       _ptr(image), n, _ptr(batch.d_offset), _ptr(batch.d_H),
                                       _ptr(batch.d_W), batch.n, _ptr(pixels), _stream(stream)))
    return pixels


def rsc_rksvd_workspace_size(h: Handle, P: int, K: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().rsc_rksvd_workspace_size(h.ptr, int(P), int(K), ctypes.byref(n)))
    return n.value


def _workspace(nbytes, dev):
    import torch
    # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)


def rsc_rksvd_update(h: Handle, xhat, atom, angle, coef, resid2, workspace=None, stream=None):
    """Dictionary update from codes under the handle's dictionary; returns device
    (d_new [M, B] float32, usage [M] int32, reset [M] int32)."""
    import torch
    P, K = atom.shape
    for t, dt in ((xhat, torch.float32), (atom, torch.int32), (angle, torch.int32), (coef, torch.float32),
                  (resid2, torch.float32)):
        if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("device contiguous tensors of the documented dtypes expected")
    if xhat.shape != (P, h.B) or resid2.shape != (P,):
        raise ValueError("shape mismatch")
    nbytes = rsc_rksvd_workspace_size(h, P, K)
    ws = workspace if workspace is not None else _workspace(nbytes, xhat.device)
    d_new = torch.empty((h.M, h.B), dtype=torch.float32, device=xhat.device)
    usage = torch.empty((h.M,), dtype=torch.int32, device=xhat.device)
    reset = torch.empty((h.M,), dtype=torch.int32, device=xhat.device)
    _check(lib().rsc_rksvd_update(h.ptr, _ptr(xhat), int(P), int(K), _ptr(atom), _ptr(angle), _ptr(coef),
                                  _ptr(resid2), _ptr(ws), ws.numel(), _ptr(d_new), _ptr(usage), _ptr(reset),
                                  _stream(stream)))
    return d_new, usage, reset


def rsc_rksvd_train(h: Handle, xhat, d_init, R: int, K: int, n_iter: int, stream=None):
    """R-K-SVD from d_init (host [M, B]); returns (D [M, B] numpy, codes of the final
    pursuit (atom, angle, coef, resid2) on the device, coding-error history numpy)."""
    import torch
    d_init = np.ascontiguousarray(d_init, dtype=np.float32)
    M, B = d_init.shape
    P = xhat.shape[0]
    if xhat.dtype != torch.float32 or not xhat.is_contiguous() or xhat.shape != (P, h.B) or B != h.B:
        raise ValueError("xhat must be device [P, B] float32 and d_init [M, B]")
    rsc_set_dictionary(h, d_init, R, stream)
    ws = _workspace(rsc_rksvd_workspace_size(h, P, K), xhat.device)
    dev = xhat.device
    atom = torch.empty((P, K), dtype=torch.int32, device=dev)
    angle = torch.empty((P, K), dtype=torch.int32, device=dev)
    coef = torch.empty((P, K), dtype=torch.float32, device=dev)
    resid2 = torch.empty((P,), dtype=torch.float32, device=dev)
    d_out = np.empty_like(d_init)
    hist = np.zeros(n_iter + 1)
    _check(lib().rsc_rksvd_train(h.ptr, _ptr(xhat), int(P), int(K), int(n_iter),
                                 d_init.ctypes.data_as(ctypes.c_void_p), int(M), int(R), _ptr(ws), ws.numel(),
                                 _ptr(atom), _ptr(angle), _ptr(coef), _ptr(resid2),
                                 d_out.ctypes.data_as(ctypes.c_void_p), hist.ctypes.data_as(ctypes.c_void_p),
                                 _stream(stream)))
    return d_out, (atom, angle, coef, resid2), hist


def rsc_precision_stats(h: Handle, reset: bool = False) -> dict:
    """Counters of a BF16 / FP16 handle's encoder (blocking)."""
    out = (ctypes.c_int64 * 4)()
    _check(lib().rsc_precision_stats(h.ptr, out, 1 if reset else 0))
    return {"steps_rescored": out[0], "candidates": out[1], "max_candidates": out[2], "fp64_solves": out[3]}


def rsc_sync(h: Handle | None = None, stream=None):
    """Waits for the stream; raises on a failed kernel or a sticky fault of h."""
    _check(lib().rsc_sync(None if h is None else h.ptr, _stream(stream)))


def rsc_last_error(h: Handle | None = None) -> str:
    return lib().rsc_last_error(None if h is None else h.ptr).decode()


# ------------------------------------------------------------------ texture classifier
def rsc_classify_workspace_size(P: int, K: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().rsc_classify_workspace_size(int(P), int(K), ctypes.byref(n)))
    return n.value


def rsc_classify(handles, xhat, K: int, workspace=None, out=None, stream=None):
    """Labels of the patches against the class dictionaries of `handles` (one per class).
    Returns (label [P] int32, sse [P] f32)."""
    import torch
    handles = list(handles)
    if not handles:
        raise ValueError("need at least one class handle")
    P = xhat.shape[0]
    _dev(xhat, torch.float32, "xhat", (P, handles[0].B))
    nbytes = rsc_classify_workspace_size(P, K)
    ws = workspace if workspace is not None else _workspace(nbytes, xhat.device)
    if out is None:
        out = (torch.empty(P, dtype=torch.int32, device=xhat.device),
               torch.empty(P, dtype=torch.float32, device=xhat.device))
    label, sse = out
    _dev(label, torch.int32, "label", (P,))
    _dev(sse, torch.float32, "sse", (P,))
    arr = (ctypes.c_void_p * len(handles))(*[h.ptr for h in handles])
    _check(lib().rsc_classify(arr, len(handles), _ptr(xhat), P, K, _ptr(ws), ws.numel(), _ptr(label),
                              _ptr(sse), _stream(stream)))
    return label, sse


def rsc_label_histogram(label, offset, C: int, out=None, stream=None):
    """Label frequencies per group; offset is a device int64 [n_groups + 1] tensor."""
    import torch
    P = label.shape[0]
    _dev(label, torch.int32, "label", (P,))
    G = offset.shape[0] - 1
    _dev(offset, torch.int64, "offset", (G + 1,))
    if out is None:
        out = torch.empty((G, C), dtype=torch.float32, device=label.device)
    _dev(out, torch.float32, "hist", (G, C))
    _check(lib().rsc_label_histogram(_ptr(label), P, _ptr(offset), G, C, _ptr(out), _stream(stream)))
    return out


def rsc_chi2_nearest(train, test, stream=None):
    """Returns (nearest [Q] int32, dist [Q] f32) for device [N, C] / [Q, C] float32 histograms."""
    import torch
    N, C = train.shape
    Q = test.shape[0]
    _dev(train, torch.float32, "train", (N, C))
    _dev(test, torch.float32, "test", (Q, C))
    nearest = torch.empty(Q, dtype=torch.int32, device=test.device)
    dist = torch.empty(Q, dtype=torch.float32, device=test.device)
    _check(lib().rsc_chi2_nearest(_ptr(train), N, _ptr(test), Q, C, _ptr(nearest), _ptr(dist), _stream(stream)))
    return nearest, dist


# ------------------------------------------------------------------ patch rotation
class RotationPlan:
    """Rotation of N x N patches by theta: interpolated (mode "nearest" or "bicubic"), or
    through a handle's steerable basis in one pass (RotationPlan.steer, 11x11)."""

    def __init__(self, N: int, theta: float, mode: str = "bicubic"):
        m = {"nearest": 0, "bicubic": 1}[mode]
        ptr = ctypes.c_void_p()
        _check(lib().rsc_rotation_plan_create(int(N), float(theta), m, ctypes.byref(ptr)))
        self.ptr, self.N, self.theta, self.mode = ptr, int(N), float(theta), mode

    @classmethod
    def steer(cls, h: "Handle", theta: float) -> "RotationPlan":
        """Phi S_theta Phi^+ of the handle's basis as one operator (rsc_rotation_plan_create_steer)."""
        ptr = ctypes.c_void_p()
        _check(lib().rsc_rotation_plan_create_steer(h.ptr, float(theta), ctypes.byref(ptr)))
        plan = cls.__new__(cls)
        plan.ptr, plan.N, plan.theta, plan.mode = ptr, h.N, float(theta), "steer"
        return plan

    def close(self):
        if self.ptr:
            lib().rsc_rotation_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rsc_rotate_interp(plan: RotationPlan, patches, out=None, stream=None):
    import torch
    P = patches.shape[0]
    _dev(patches, torch.float32, "patches", (P, plan.N, plan.N))
    if out is None:
        out = torch.empty_like(patches)
    _dev(out, torch.float32, "out", (P, plan.N, plan.N))
    _check(lib().rsc_rotate_interp(plan.ptr, _ptr(patches), P, _ptr(out), _stream(stream)))
    return out


def rsc_steer(h: Handle, xhat, theta0: float = 0.0, theta=None, out=None, stream=None):
    """S_theta x_hat: one angle theta0 for every patch, or a device float32 [P] of angles."""
    import torch
    P = xhat.shape[0]
    _dev(xhat, torch.float32, "xhat", (P, h.B))
    if theta is not None:
        _dev(theta, torch.float32, "theta", (P,))
    if out is None:
        out = torch.empty_like(xhat)
    _dev(out, torch.float32, "out", (P, h.B))
    _check(lib().rsc_steer(h.ptr, _ptr(xhat), P, _ptr(theta), float(theta0), _ptr(out), _stream(stream)))
    return out


def rsc_synthesize_hat(h: Handle, xhat, out=None, stream=None):
    """Phi x_hat on the N x N grid, zero off the disk."""
    import torch
    P = xhat.shape[0]
    _dev(xhat, torch.float32, "xhat", (P, h.B))
    if out is None:
        out = torch.empty((P, h.N, h.N), dtype=torch.float32, device=xhat.device)
    _dev(out, torch.float32, "pixels", (P, h.N, h.N))
    _check(lib().rsc_synthesize_hat(h.ptr, _ptr(xhat), P, _ptr(out), _stream(stream)))
    return out

