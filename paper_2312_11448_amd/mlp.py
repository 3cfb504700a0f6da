"""Binding of the mixing-correction surrogate network (argument marshalling
only; the network runs in the HIP library)."""
import torch

from . import _abi as A


class Mlp:
    """The 8-64-64-1 ReLU network on one device and stream."""

    def __init__(self, params, device="cuda", stream=None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self.h = A.mc_lya_mlp_create([float(x) for x in params], self.stream)

    def params(self):
        return A.mc_lya_mlp_get_params(self.h)

    def set_envelope(self, lo, hi):
        A.mc_lya_mlp_set_envelope(self.h, lo, hi)

    def forward(self, features, outside=False, count=False):
        """features: float32 [n, 8] contiguous tensor on the device. Returns y
        (and the uint8 outside-envelope flags, and their count, if asked)."""
        f = features.contiguous()
        n = f.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        flags = torch.empty(n, dtype=torch.uint8, device=self.device) if outside else None
        c = A.mc_lya_mlp_forward(self.h, f.data_ptr(), n, y.data_ptr(),
                                 flags.data_ptr() if flags is not None else None, count)
        out = [y]
        if outside:
            out.append(flags)
        if count:
            out.append(c)
        return out[0] if len(out) == 1 else tuple(out)

    def correction(self, features, fallback=None):
        """The mixing correction M per cell, with the Monte Carlo's M
        (`fallback`, float32 [n]) taken where the features leave the training
        envelope. Returns (M, y, outside flags, number outside)."""
        f = features.contiguous()
        n = f.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        m = torch.empty_like(y)
        flags = torch.empty(n, dtype=torch.uint8, device=self.device)
        fb = None
        if fallback is not None:
            fallback = fallback.contiguous()
            assert fallback.dtype == torch.float32 and fallback.shape[0] == n
            fb = fallback.data_ptr()
        c = A.mc_lya_mlp_correction(self.h, f.data_ptr(), n, fb, y.data_ptr(), m.data_ptr(), flags.data_ptr(), True)
        return m, y, flags, c

    def gradient(self, features, targets, weights):
        """(gradient [4801] as a list, loss) of the weighted MSE."""
        return A.mc_lya_mlp_gradient(self.h, features.contiguous().data_ptr(), targets.contiguous().data_ptr(),
                                     weights.contiguous().data_ptr(), features.shape[0])

    def train_step(self, features, targets, weights, lr, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        return A.mc_lya_mlp_train_step(self.h, features.data_ptr(), targets.data_ptr(), weights.data_ptr(),
                                       features.shape[0], lr, beta1, beta2, eps, want_loss)

    def train_steps(self, features, targets, weights, idx, lrs, beta1=0.9, beta2=0.999, eps=1e-8,
                    want_losses=False):
        """len(lrs) training steps in one call: step s on the cells
        idx[s] (int64 [steps][batch] device tensor) of the training set.
        Returns each step's loss if asked."""
        assert idx.dtype == torch.int64 and idx.dim() == 2 and idx.shape[0] == len(lrs)
        f = features.contiguous()
        t = targets.contiguous()
        w = weights.contiguous()
        i = idx.contiguous()
        return A.mc_lya_mlp_train_steps(self.h, f.data_ptr(), t.data_ptr(), w.data_ptr(), f.shape[0], i.data_ptr(),
                                        i.shape[1], lrs, beta1, beta2, eps, want_losses)

    def close(self):
        if self.h:
            A.mc_lya_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
