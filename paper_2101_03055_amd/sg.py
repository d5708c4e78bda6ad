"""Python binding of include/sg.h (CNN surrogate; argument marshalling only)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lb as _lb

SG_LAYERS, SG_IN_PARAMS, SG_OUTPUTS = 6, 5, 4


class sg_config(C.Structure):
    _fields_ = [("batch", C.c_int32), ("height", C.c_int32), ("width", C.c_int32), ("reserved", C.c_int32),
                ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


_done = False


def lib():
    global _done
    L = _lb.lib()
    if not _done:
        vp, sz, i32, i64, st = C.c_void_p, C.c_size_t, C.c_int32, C.c_int64, C.c_int
        pc = C.POINTER(sg_config)
        pi = C.POINTER(C.c_int32)
        sig = {
            "sg_layer_info": [i32, pi, pi, pi, pi],
            "sg_param_count": [C.POINTER(i64), C.POINTER(i64)],
            "sg_workspace_bytes": [pc, C.POINTER(sz)],
            "sg_create": [pc, vp, sz, vp, C.POINTER(vp)],
            "sg_set_weights": [vp, vp],
            "sg_get_weights": [vp, vp],
            "sg_gradients": [vp, vp, vp, vp, vp, vp],
            "sg_train_step": [vp, vp, vp, vp, vp],
            "sg_train_epochs": [vp, vp, vp, i32, i32, C.c_uint64, vp],
            "sg_predict": [vp, vp, i32, vp],
            "sg_layer_output": [vp, i32, vp],
            "sg_layer_input": [vp, i32, vp],
            "sg_conv": [vp, i32, i32, i32, vp, vp, vp, vp],
            "sg_weight_grad": [vp, i32, i32, vp, vp, vp, vp],
            "sg_free": [vp],
            "sg_smooth": [vp, vp, i32, i32, i32, vp],
            "sg_destagger": [vp, i32, i32, i32, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.sg_last_error.restype = C.c_char_p
        _done = True
    return L


def _check(status):
    if status != 0:
        raise _lb.LBError(status, lib().sg_last_error().decode())


def layer_info(l: int):
    v = [C.c_int32() for _ in range(4)]
    _check(lib().sg_layer_info(l, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)  # cin, cout, cin_pad, cout_pad


def param_count():
    p, r = C.c_int64(), C.c_int64()
    _check(lib().sg_param_count(C.byref(p), C.byref(r)))
    return p.value, r.value


def unpack(vec):
    """Packed FP32 vector -> list of (w[co, tap, ci], b[co]) over padded channels."""
    out, off = [], 0
    for l in range(SG_LAYERS):
        _, _, ci, co = layer_info(l)
        w = vec[off:off + co * 9 * ci].reshape(co, 9, ci)
        off += co * 9 * ci
        b = vec[off:off + co]
        off += co
        out.append((w, b))
    return out


def init_weights(seed: int = 0, gain: float = 1.0):
    """Seeded He-style initialisation of the real channels; padding stays 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    packed, _ = param_count()
    vec = np.zeros(packed, dtype=np.float32)
    off = 0
    for l in range(SG_LAYERS):
        cin, cout, ci, co = layer_info(l)
        w = np.zeros((co, 9, ci), dtype=np.float32)
        std = gain * np.sqrt(2.0 / (9 * cin)) if l + 1 < SG_LAYERS else gain * np.sqrt(1.0 / (9 * cin))
        w[:cout, :, :cin] = rng.standard_normal((cout, 9, cin)) * std
        vec[off:off + co * 9 * ci] = w.ravel()
        off += co * 9 * ci + co
    return vec


def smooth(d_in, d_out, stream=None):
    """[1 2 1] x [1 2 1] filter of every [..., H, W] plane of a CUDA float32 tensor."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(d_in.device)
    H, W = d_in.shape[-2], d_in.shape[-1]
    planes = d_in.numel() // (H * W)
    _check(lib().sg_smooth(C.c_void_p(d_in.data_ptr()), C.c_void_p(d_out.data_ptr()), planes, H, W,
                           C.c_void_p(s.cuda_stream)))


def destagger(d_fields, stream=None):
    """Remove the lattice-staggered velocity parts of CUDA float32 fields [n, 4, H, W] in place."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(d_fields.device)
    n, c, H, W = d_fields.shape
    assert c == 4 and d_fields.dtype == torch.float32 and d_fields.is_contiguous()
    _check(lib().sg_destagger(C.c_void_p(d_fields.data_ptr()), n, H, W, C.c_void_p(s.cuda_stream)))


class Surrogate:
    def __init__(self, batch: int, height: int, width: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 device: str = "cuda:0"):
        import torch

        self.cfg = sg_config(batch, height, width, 0, lr, beta1, beta2, eps)
        n = C.c_size_t()
        _check(lib().sg_workspace_bytes(C.byref(self.cfg), C.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.workspace.device)
        h = C.c_void_p()
        _check(lib().sg_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()), n.value,
                               C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self.packed, self.real = param_count()

    def set_weights(self, vec):
        vec = np.ascontiguousarray(vec, dtype=np.float32)
        assert vec.size == self.packed
        _check(lib().sg_set_weights(self.handle, vec.ctypes.data))

    def get_weights(self):
        out = np.empty(self.packed, dtype=np.float32)
        _check(lib().sg_get_weights(self.handle, out.ctypes.data))
        return out

    def gradients(self, d_params, d_fields, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        loss = C.c_float()
        g = np.empty(self.packed, dtype=np.float32)
        _check(lib().sg_gradients(self.handle, C.c_void_p(d_params.data_ptr()), C.c_void_p(d_fields.data_ptr()),
                                  idx.ctypes.data, C.byref(loss), g.ctypes.data))
        return loss.value, g

    def train_step(self, d_params, d_fields, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        loss = C.c_float()
        _check(lib().sg_train_step(self.handle, C.c_void_p(d_params.data_ptr()), C.c_void_p(d_fields.data_ptr()),
                                   idx.ctypes.data, C.byref(loss)))
        return loss.value

    def train_epochs(self, d_params, d_fields, n: int, epochs: int, seed: int = 0):
        losses = np.empty(max(epochs, 1), dtype=np.float32)
        _check(lib().sg_train_epochs(self.handle, C.c_void_p(d_params.data_ptr()), C.c_void_p(d_fields.data_ptr()),
                                     int(n), int(epochs), int(seed), losses.ctypes.data))
        return losses[:epochs]

    def predict(self, d_params, n: int, d_out):
        _check(lib().sg_predict(self.handle, C.c_void_p(d_params.data_ptr()), int(n), C.c_void_p(d_out.data_ptr())))

    def layer_output(self, l: int):
        _, _, _, co = layer_info(l)
        out = np.empty((self.cfg.batch, self.cfg.height, self.cfg.width, co), dtype=np.float32)
        _check(lib().sg_layer_output(self.handle, l, out.ctypes.data))
        return out

    def layer_input(self, l: int):
        _, _, ci, _ = layer_info(l)
        out = np.empty((self.cfg.batch, self.cfg.height, self.cfg.width, ci), dtype=np.float32)
        _check(lib().sg_layer_input(self.handle, l, out.ctypes.data))
        return out

    def conv(self, layer: int, mode: int, nb: int, d_in, d_out, d_z=None, d_zprev=None):
        """One convolution of the training pass on CUDA tensors (sg_conv): bf16
        tensors d_in/d_out, float32 d_z (forward) or d_zprev (data gradient)."""
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        _check(lib().sg_conv(self.handle, layer, mode, nb, ptr(d_in), ptr(d_zprev), ptr(d_z), ptr(d_out)))

    def weight_grad(self, layer: int, nb: int, d_g, d_x, d_dw, d_db):
        """Weight and bias gradients of one layer on CUDA tensors (sg_weight_grad)."""
        _check(lib().sg_weight_grad(self.handle, layer, nb, C.c_void_p(d_g.data_ptr()), C.c_void_p(d_x.data_ptr()),
                                    C.c_void_p(d_dw.data_ptr()), C.c_void_p(d_db.data_ptr())))

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().sg_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
