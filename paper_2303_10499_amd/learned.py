"""Python binding of the learned-preconditioner network (include/gea_learned.h).

Argument marshalling only: forward, backward and Adam run in the library's
bfloat16 matrix-core kernels; torch supplies the workspace and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import gea


def _lib():
    L = gea.lib()
    if not getattr(L, "_learned_bound", False):
        P, vp = C.POINTER, C.c_void_p
        L.gea_cnn_param_count.argtypes = [C.c_int32, P(C.c_int64)]
        L.gea_cnn_workspace_bytes.argtypes = [C.c_int32] * 5 + [P(C.c_size_t)]
        L.gea_cnn_create.argtypes = [C.c_int32] * 5 + [vp, vp, C.c_size_t, P(vp)]
        L.gea_cnn_set_params.argtypes = [vp, vp, C.c_int]
        L.gea_cnn_get_params.argtypes = [vp, vp, C.c_int]
        L.gea_cnn_forward.argtypes = [vp, vp, vp, C.c_int]
        L.gea_cnn_backward.argtypes = [vp, vp, C.c_int, C.c_int32, P(C.c_double)]
        L.gea_cnn_get_grads.argtypes = [vp, vp, C.c_int]
        L.gea_cnn_adam.argtypes = [vp, C.c_float, C.c_float, C.c_int32]
        L.gea_cnn_activation.argtypes = [vp, C.c_int32, vp, C.c_int]
        L.gea_cnn_destroy.argtypes = [vp]
        L.gea_cnn_destroy.restype = None
        L.gea_load_weights.argtypes = [vp, vp, C.c_int]
        L.gea_make_pair.argtypes = [vp, C.c_double, vp, vp, vp, P(C.c_double), C.c_int]
        L.gea_learned_apply.argtypes = [vp, vp, vp, P(C.c_double), C.c_int]
        L.gea_learned_activation.argtypes = [vp, C.c_int32, vp, C.c_int]
        for n in ("gea_cnn_param_count", "gea_cnn_workspace_bytes", "gea_cnn_create",
                  "gea_cnn_set_params", "gea_cnn_get_params", "gea_cnn_forward",
                  "gea_cnn_backward", "gea_cnn_get_grads", "gea_cnn_adam", "gea_load_weights",
                  "gea_cnn_activation", "gea_learned_apply", "gea_learned_activation",
                  "gea_make_pair"):
            getattr(L, n).restype = C.c_int
        L._learned_bound = True
    return L


def weights_file(ndim: int) -> str:
    """trained weights shipped with the package (written by train.py)"""
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", f"net{ndim}d.npy")


def param_count(ndim: int) -> int:
    n = C.c_int64(0)
    rc = _lib().gea_cnn_param_count(ndim, C.byref(n))
    if rc != gea.OK:
        raise gea.GeaError(rc, "gea_cnn_param_count")
    return n.value


def layer_shapes(ndim: int):
    """(C_out, taps, C_in) of W and C_out of b, per layer, in packed order"""
    nt = 3 ** ndim
    shapes = [(16, 2), (32, 16), (64, 32), (32, 96), (16, 48), (1, 16)]
    return [((co, nt, ci), co) for co, ci in shapes]


def pack(params) -> np.ndarray:
    """list of (W, b) -> packed FP32 vector"""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                           np.asarray(b, np.float32).ravel()]) for W, b in params])


def unpack(vec, ndim: int):
    out, off = [], 0
    for wshape, nb in layer_shapes(ndim):
        nw = int(np.prod(wshape))
        out.append((np.asarray(vec[off:off + nw]).reshape(wshape), np.asarray(vec[off + nw:off + nw + nb])))
        off += nw + nb
    return out


def _ptr(a):
    if isinstance(a, np.ndarray):
        assert a.dtype == np.float32 and a.flags.c_contiguous
        return a.ctypes.data, gea.HOST
    assert a.dtype.__str__() == "torch.float32" and a.is_contiguous()
    return a.data_ptr(), (gea.DEVICE if a.is_cuda else gea.HOST)


class Net:
    """One network instance on an nx x ny x nz grid (ny = 1 in 2D)."""

    def __init__(self, ndim, nx, ny, nz, train=True, device="cuda:0"):
        import torch
        self.torch = torch
        self.L = _lib()
        self.ndim, self.shape = ndim, (nx, ny, nz)
        self.npix = nx * ny * nz
        nb = C.c_size_t(0)
        rc = self.L.gea_cnn_workspace_bytes(ndim, nx, ny, nz, int(train), C.byref(nb))
        if rc != gea.OK:
            raise gea.GeaError(rc, "gea_cnn_workspace_bytes: dimensions must be multiples of 4")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(torch.device(device))
        h = C.c_void_p()
        rc = self.L.gea_cnn_create(ndim, nx, ny, nz, int(train), C.c_void_p(self.stream.cuda_stream),
                                   C.c_void_p(self.ws.data_ptr()), nb.value, C.byref(h))
        if rc != gea.OK:
            raise gea.GeaError(rc, "gea_cnn_create")
        self.h = h
        self.nparams = param_count(ndim)

    def close(self):
        if getattr(self, "h", None):
            self.L.gea_cnn_destroy(self.h)
            self.h = None

    __del__ = close

    def _ok(self, rc, what):
        if rc != gea.OK:
            raise gea.GeaError(rc, what)

    def set_params(self, vec):
        vec = np.ascontiguousarray(vec, dtype=np.float32) if isinstance(vec, np.ndarray) else vec
        p, k = _ptr(vec)
        self._ok(self.L.gea_cnn_set_params(self.h, C.c_void_p(p), k), "set_params")

    def get_params(self):
        out = np.empty(self.nparams, np.float32)
        self._ok(self.L.gea_cnn_get_params(self.h, C.c_void_p(out.ctypes.data), gea.HOST), "get_params")
        return out

    def forward(self, x, y=None):
        """x: npix x 2 FP32 (numpy or torch); returns y (npix)"""
        if y is None:
            y = np.empty(self.npix, np.float32) if isinstance(x, np.ndarray) else \
                self.torch.empty(self.npix, dtype=self.torch.float32, device=x.device)
        xp, k = _ptr(x)
        yp, _ = _ptr(y)
        self._ok(self.L.gea_cnn_forward(self.h, C.c_void_p(xp), C.c_void_p(yp), k), "forward")
        return y

    def backward(self, t, accumulate=False):
        tp, k = _ptr(t)
        loss = C.c_double(0.0)
        self._ok(self.L.gea_cnn_backward(self.h, C.c_void_p(tp), k, int(accumulate), C.byref(loss)), "backward")
        return loss.value

    def get_grads(self):
        out = np.empty(self.nparams, np.float32)
        self._ok(self.L.gea_cnn_get_grads(self.h, C.c_void_p(out.ctypes.data), gea.HOST), "get_grads")
        return out

    ACT = {"xin": (0, 0, 8), "e0": (1, 0, 16), "p0": (2, 1, 16), "e1": (3, 1, 32),
           "p1": (4, 2, 32), "e2": (5, 2, 64), "c1": (6, 1, 96), "d1": (7, 1, 32),
           "c0": (8, 0, 48), "d0": (9, 0, 16)}

    def activation(self, name):
        """an activation of the last forward pass (FP32, grid shape + channels)"""
        which, level, ch = self.ACT[name]
        nx, ny, nz = self.shape
        sp = (nz >> level, nx >> level) if self.ndim == 2 else (nz >> level, ny >> level, nx >> level)
        out = np.empty(int(np.prod(sp)) * ch, np.float32)
        self._ok(self.L.gea_cnn_activation(self.h, which, C.c_void_p(out.ctypes.data), gea.HOST), "activation")
        return out.reshape(sp + (ch,))

    def adam(self, lr, step, grad_scale=1.0):
        self._ok(self.L.gea_cnn_adam(self.h, float(lr), float(grad_scale), int(step)), "adam")


def solver_apply(S, r):
    """The learned solver's network application on the FP32 residual r (host
    array of S.nc values) of solver S's last assembled system: (z, s) with
    s = max |r| and z = s * net(r/s, c/diag)."""
    r = np.ascontiguousarray(r, dtype=np.float32)
    z = np.empty(S.nc, np.float32)
    s = C.c_double(0.0)
    rc = _lib().gea_learned_apply(S.ctx, C.c_void_p(r.ctypes.data), C.c_void_p(z.ctypes.data),
                                  C.byref(s), gea.HOST)
    if rc != gea.OK:
        raise gea.GeaError(rc, S.L.gea_last_error(S.ctx).decode())
    return z, s.value


def solver_activation(S, name):
    """an activation of solver S's network after solver_apply (FP32, grid
    shape + channels); 'x2' gives the two input channels"""
    if name == "x2":
        which, level, ch = 0, 0, 2
    else:
        which, level, ch = Net.ACT[name]
    m = S.mesh
    sp = (m.nz >> level, m.nx >> level) if S.ndim == 2 else (m.nz >> level, m.ny >> level, m.nx >> level)
    out = np.empty(int(np.prod(sp)) * ch, np.float32)
    rc = _lib().gea_learned_activation(S.ctx, which, C.c_void_p(out.ctypes.data), gea.HOST)
    if rc != gea.OK:
        raise gea.GeaError(rc, S.L.gea_last_error(S.ctx).decode())
    return out.reshape(sp + (ch,))
