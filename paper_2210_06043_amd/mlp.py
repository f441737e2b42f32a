"""ctypes binding of the surrogate C-ABI (``include/capib_mlp.h``): the
perceptron that predicts drag, lift and bond-rupture hazard of an adhered
particle.  Argument marshalling only; every computation runs in the HIP
kernels of libcapib.so."""
import ctypes as C

import numpy as np

from . import capib

IN, HIDDEN, OUT, N_PARAMS = 37, 256, 3, 207875
_P = C.c_void_p
_fp = C.POINTER(C.c_float)

SIGNATURES = {
    "capib_mlp_create": (C.c_int, [C.c_int32, _P, C.POINTER(_P)]),
    "capib_mlp_workspace_bytes": (C.c_size_t, [_P]),
    "capib_mlp_bind_workspace": (C.c_int, [_P, _P, C.c_size_t]),
    "capib_mlp_set_params": (C.c_int, [_P, _fp]),
    "capib_mlp_get_params": (C.c_int, [_P, _fp]),
    "capib_mlp_forward": (C.c_int, [_P, _P, C.c_int32, _P]),
    "capib_mlp_loss_grad": (C.c_int, [_P, _P, _P, C.c_int32, C.POINTER(C.c_double), _fp]),
    "capib_mlp_adam_step": (C.c_int, [_P, C.c_float]),
    "capib_mlp_last_error": (C.c_char_p, [_P]),
    "capib_mlp_destroy": (None, [_P]),
}
_bound = False


def _lib():
    global _bound
    L = capib.load_library()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _bound = True
    return L


class Surrogate:
    """The surrogate on the current HIP device, for batches of up to
    max_batch samples; inputs, targets and outputs are torch tensors on the
    device (float32, contiguous)."""

    def __init__(self, max_batch, stream=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the surrogate runs only on the GPU")
        self.torch = torch
        self.L = _lib()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.h = _P()
        st = self.L.capib_mlp_create(int(max_batch), _P(self.stream.cuda_stream), C.byref(self.h))
        if st != capib.CAPIB_OK:
            raise capib.CapibError(st, "capib_mlp_create rejected the batch size")
        nbytes = self.L.capib_mlp_workspace_bytes(self.h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._check(self.L.capib_mlp_bind_workspace(self.h, _P((self.workspace.data_ptr() + 255) & ~255), nbytes))
        self.max_batch = int(max_batch)

    def _check(self, st):
        if st != capib.CAPIB_OK:
            raise capib.CapibError(st, self.L.capib_mlp_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.L.capib_mlp_destroy(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, cols):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected [n][{cols}]")
        return t

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        if v.size != N_PARAMS:
            raise ValueError(f"{N_PARAMS} parameters expected")
        self._check(self.L.capib_mlp_set_params(self.h, v.ctypes.data_as(_fp)))

    def get_params(self):
        v = np.zeros(N_PARAMS, dtype=np.float32)
        self._check(self.L.capib_mlp_get_params(self.h, v.ctypes.data_as(_fp)))
        return v

    def forward(self, x):
        x = self._dev(x, IN)
        y = self.torch.empty((x.shape[0], OUT), dtype=self.torch.float32, device=self.device)
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self._check(self.L.capib_mlp_forward(self.h, _P(x.data_ptr()), x.shape[0], _P(y.data_ptr())))
        x.record_stream(self.stream)      # the caller's allocator must not reuse x before the kernels read it
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return y

    def loss_grad(self, x, t, want_grads=False):
        x, t = self._dev(x, IN), self._dev(t, OUT)
        loss = C.c_double()
        g = np.zeros(N_PARAMS, dtype=np.float32) if want_grads else None
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self._check(self.L.capib_mlp_loss_grad(self.h, _P(x.data_ptr()), _P(t.data_ptr()), x.shape[0],
                                               C.byref(loss), g.ctypes.data_as(_fp) if g is not None else None))
        x.record_stream(self.stream)
        t.record_stream(self.stream)
        return loss.value, g

    def train_step(self, x, t, lr):
        """Gradients on a batch and one Adam update (no host sync)."""
        x, t = self._dev(x, IN), self._dev(t, OUT)
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self._check(self.L.capib_mlp_loss_grad(self.h, _P(x.data_ptr()), _P(t.data_ptr()), x.shape[0], None, None))
        x.record_stream(self.stream)
        t.record_stream(self.stream)
        self._check(self.L.capib_mlp_adam_step(self.h, float(lr)))

    def adam_step(self, lr):
        self._check(self.L.capib_mlp_adam_step(self.h, float(lr)))

    def synchronize(self):
        self.stream.synchronize()
