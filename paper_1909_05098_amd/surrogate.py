"""Thin ctypes binding of the surrogate entry points (fedfem_surrogate.h).

Argument marshalling only: the network's forward and backward passes, the
loss, Adam, rasterisation and resampling run in the library's HIP kernels.
Device memory is held in torch tensors (BF16 tensors are passed by pointer).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import fedfem as ff

IN_CHANNELS = 8
LAYERS = [("e1a", 8, 32), ("e1b", 32, 32), ("e2a", 32, 64), ("e2b", 64, 64),
          ("e3a", 64, 128), ("e3b", 128, 128), ("d2a", 192, 64), ("d2b", 64, 64),
          ("d1a", 96, 32), ("d1b", 32, 32)]
LEVEL = [0, 0, 1, 1, 2, 2, 1, 1, 0, 0]

_P = C.c_void_p
_SIGS = {
    "fedsur_create": (C.c_int, [C.c_int32, C.c_int32, C.c_uint64, _P]),
    "fedsur_destroy": (C.c_int, [_P]),
    "fedsur_set_stream": (C.c_int, [_P, _P]),
    "fedsur_param_count": (C.c_int, [_P, _P]),
    "fedsur_get_params": (C.c_int, [_P, _P]),
    "fedsur_set_params": (C.c_int, [_P, _P]),
    "fedsur_get_grads": (C.c_int, [_P, _P]),
    "fedsur_forward": (C.c_int, [_P, C.c_int32, _P, _P]),
    "fedsur_loss_backward": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
    "fedsur_adam_step": (C.c_int, [_P, C.c_float]),
    "fedsur_read_activation": (C.c_int, [_P, C.c_int32, _P]),
    "fedsur_rasterize": (C.c_int, [C.c_int32, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "fedsur_target": (C.c_int, [C.c_int32, C.c_int32, _P, _P, _P, _P, C.c_float, C.c_float, _P,
                                _P, _P]),
    "fedsur_decode": (C.c_int, [C.c_int32, C.c_int32, _P, _P, C.c_float, _P, _P]),
    "fedsur_max_error": (C.c_int, [C.c_int32, C.c_int32, _P, _P, _P, _P, _P]),
    "fedfem_resample": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
}
_bound = False

# fedsur_sample: one record of 12 doubles per sample
SAMPLE_FIELDS = ("cx", "cy", "cz", "sigma", "q0", "k0", "omega_b", "ax", "ay", "az",
                 "hmesh", "reserved")


def lib():
    global _bound
    L = ff.load()
    if not _bound:
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _bound = True
    return L


def exported_symbols():
    return sorted(_SIGS)


def _check(rc, what):
    if rc != ff.OK:
        raise ff.FedFemError(rc, f"{what}: " + lib().fedfem_strerror(rc).decode())


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def param_layout():
    """[(name, offset, shape)] of the FP32 parameter vector."""
    out, off = [], 0
    for name, ci, co in LAYERS:
        out.append((name + ".w", off, (co, 3, 3, 3, ci)))
        off += co * 27 * ci
        out.append((name + ".b", off, (co,)))
        off += co
    out.append(("head.w", off, (32,)))
    out.append(("head.b", off + 32, (1,)))
    return out


def unflatten(vec):
    return {n: np.asarray(vec[o:o + int(np.prod(s))]).reshape(s)
            for n, o, s in param_layout()}


def flatten(P):
    parts = [np.asarray(P[n], dtype=np.float64).reshape(-1) for n, _, _ in param_layout()]
    return np.concatenate(parts)


class Net:
    """The 3-level encoder-decoder on a G^3 grid (device resident)."""

    def __init__(self, grid, batch_max, seed=0):
        self._L = lib()
        self._n = C.c_void_p()
        self.G = int(grid)
        self.batch_max = int(batch_max)
        _check(self._L.fedsur_create(self.G, self.batch_max, C.c_uint64(seed),
                                     C.byref(self._n)), "fedsur_create")
        cnt = C.c_int64()
        _check(self._L.fedsur_param_count(self._n, C.byref(cnt)), "fedsur_param_count")
        self.n_params = cnt.value

    def close(self):
        if self._n:
            self._L.fedsur_destroy(self._n)
            self._n = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        """Run the network's kernels on `stream` (a HIP stream handle, e.g.
        torch.cuda.current_stream().cuda_stream; 0 = the legacy default
        stream)."""
        _check(self._L.fedsur_set_stream(self._n, C.c_void_p(stream or None)),
               "fedsur_set_stream")

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self._L.fedsur_get_params(self._n, out.ctypes.data_as(_P)), "fedsur_get_params")
        return out

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.n_params
        _check(self._L.fedsur_set_params(self._n, v.ctypes.data_as(_P)), "fedsur_set_params")

    def get_grads(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self._L.fedsur_get_grads(self._n, out.ctypes.data_as(_P)), "fedsur_get_grads")
        return out

    def forward(self, x, y):
        """x: bf16 cuda tensor [B, G, G, G, 8]; y: float32 cuda tensor [B, G, G, G]."""
        _check(self._L.fedsur_forward(self._n, x.shape[0], _dptr(x), _dptr(y)), "fedsur_forward")

    def loss_backward(self, x, target, mask):
        loss = C.c_float()
        _check(self._L.fedsur_loss_backward(self._n, x.shape[0], _dptr(x), _dptr(target),
                                            _dptr(mask), C.byref(loss)), "fedsur_loss_backward")
        return loss.value

    def adam_step(self, lr):
        _check(self._L.fedsur_adam_step(self._n, C.c_float(lr)), "fedsur_adam_step")

    def activation(self, layer, batch):
        name, ci, co = LAYERS[layer]
        g = self.G >> LEVEL[layer]
        out = np.empty((batch, g, g, g, co), dtype=np.float32)
        _check(self._L.fedsur_read_activation(self._n, layer, out.ctypes.data_as(_P)),
               "fedsur_read_activation")
        return out


def _stream(stream):
    return None if not stream else C.c_void_p(stream)


def rasterize(grid, frame, samples, phys, x, prior, scale, stream=None):
    """Network input x (bf16 cuda [B, G, G, G, 8]), prior (float32 cuda
    [B, G, G, G] or None) and scale (float32 cuda [B]) from samples
    (float64 cuda [B, 12], fields SAMPLE_FIELDS) and phys = (rho0, c0,
    rho_b c_b, t_heat)."""
    fr = np.ascontiguousarray(frame, dtype=np.float64)
    ph = np.ascontiguousarray(phys, dtype=np.float64)
    assert samples.shape[-1] == len(SAMPLE_FIELDS) and ph.size == 4
    _check(lib().fedsur_rasterize(int(grid), fr.ctypes.data_as(_P), samples.shape[0],
                                  _dptr(samples), ph.ctypes.data_as(_P), _dptr(x),
                                  None if prior is None else _dptr(prior), _dptr(scale),
                                  _stream(stream)), "fedsur_rasterize")


def target(grid, prior, scale, T, mask, T_a, out, weight, focus=0.0, stream=None):
    """out = (T - T_a - prior) / scale inside mask, weight = mask (1 +
    focus prior / scale) (cuda)."""
    _check(lib().fedsur_target(int(grid), prior.shape[0], _dptr(prior), _dptr(scale), _dptr(T),
                               _dptr(mask), C.c_float(T_a), C.c_float(focus), _dptr(out),
                               _dptr(weight), _stream(stream)), "fedsur_target")


def decode(grid, prior, scale, T_a, y, stream=None):
    """y <- T_a + prior + scale * y in place (cuda)."""
    _check(lib().fedsur_decode(int(grid), prior.shape[0], _dptr(prior), _dptr(scale),
                               C.c_float(T_a), _dptr(y), _stream(stream)), "fedsur_decode")


def max_error(grid, Tp, T, mask, err, stream=None):
    """err[b] = max over mask of |Tp - T| (cuda float32 [B])."""
    _check(lib().fedsur_max_error(int(grid), Tp.shape[0], _dptr(Tp), _dptr(T), _dptr(mask),
                                  _dptr(err), _stream(stream)), "fedsur_max_error")


def resample(handle, grid, frame, T_out, mask_out):
    """P1 interpolation of a handle's T at voxel centres (cuda tensors)."""
    fr = np.ascontiguousarray(frame, dtype=np.float64)
    _check(lib().fedfem_resample(handle._h, int(grid), fr.ctypes.data_as(_P), _dptr(T_out),
                                 _dptr(mask_out)), "fedfem_resample")
