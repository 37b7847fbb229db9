"""The warm-start U-Net, built from the layer calls of include/lbm_nn.h.

Architecture: 4 levels of 16, 32, 64 and 128 channels; each level two 3x3x3 ReLU
convolutions; 2x2x2 mean pooling down, nearest upsampling up, skip connections
concatenated as [skip, upsampled]; a 1x1x1 head to the output channels.  Input: 16
channels per voxel (pore mask, pore diameter / d_scale, 14 zeros).  Weights are binary32
masters with bf16 copies for the matrix cores; Adam on the masters.

This module only sequences the calls and owns the buffers (torch tensors); every layer
runs in the library's kernels.
"""
import numpy as np
import torch

from . import nn
from .nn import View

LEVELS = (16, 32, 64, 128)
C_IN = 16


def _layers(levels=LEVELS):
    L = [("enc0a", C_IN, levels[0]), ("enc0b", levels[0], levels[0])]
    for i in range(1, len(levels)):
        L += [(f"enc{i}a", levels[i - 1], levels[i]), (f"enc{i}b", levels[i], levels[i])]
    for i in range(len(levels) - 2, -1, -1):
        L += [(f"dec{i}a", levels[i] + levels[i + 1], levels[i]), (f"dec{i}b", levels[i], levels[i])]
    return L


class UNet:
    def __init__(self, n_out=5, seed=0, device="cuda"):
        self.n_out = n_out
        self.layers = _layers()
        self.off = {}
        n = 0
        for name, ci, co in self.layers:
            self.off[name + ".w"] = (n, 27 * co * ci)
            n += 27 * co * ci
            self.off[name + ".b"] = (n, co)
            n += co
        self.off["head.w"] = (n, n_out * LEVELS[0])
        n += n_out * LEVELS[0]
        self.off["head.b"] = (n, n_out)
        n += n_out
        self.n_params = n
        dev = torch.device(device)
        self.p = torch.zeros(n, dtype=torch.float32, device=dev)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.pb = torch.zeros(n, dtype=torch.bfloat16, device=dev)
        self.wt = {name: torch.zeros(27 * ci * co, dtype=torch.bfloat16, device=dev)
                   for name, ci, co in self.layers}
        self.step = 0
        self._bufs = {}
        self._init(seed)

    # ---------------------------------------------------------------- parameters
    def _init(self, seed):
        """He-normal convolution weights (input channels 2..15 of the first layer carry no
        signal and start at zero), zero biases, a small head."""
        gen = torch.Generator().manual_seed(seed)
        host = torch.zeros(self.n_params, dtype=torch.float32)
        for name, ci, co in self.layers:
            o, k = self.off[name + ".w"]
            fan = 27 * (2 if name == "enc0a" else ci)
            w = torch.randn(27, co, ci, generator=gen) * (2.0 / fan) ** 0.5
            if name == "enc0a":
                w[:, :, 2:] = 0.0
            host[o:o + k] = w.reshape(-1)
        o, k = self.off["head.w"]
        host[o:o + k] = torch.randn(k, generator=gen) * (1.0 / LEVELS[0]) ** 0.5
        self.load_flat(host.numpy())

    def load_flat(self, flat):
        flat = np.asarray(flat, np.float32)
        if flat.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters, got {flat.shape}")
        self.p.copy_(torch.from_numpy(flat))
        self._refresh()

    def _refresh(self):
        nn.lbm_nn_to_bf16(self.p, self.pb)
        self._transpose()

    def _transpose(self):
        for name, ci, co in self.layers:
            nn.lbm_nn_transpose_weights(self.w_bf(name), co, ci, self.wt[name])

    def w_bf(self, name):
        o, k = self.off[name + ".w"]
        return self.pb[o:o + k]

    def view(self, t, name):
        o, k = self.off[name]
        return t[o:o + k]

    def save(self, path):
        np.savez(path, params=self.p.cpu().numpy(), layers=np.array(
            [f"{n}:{ci}:{co}" for n, ci, co in self.layers]), n_out=self.n_out)

    @classmethod
    def load(cls, path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        net = cls(n_out=int(z["n_out"]), device=device)
        layers = [f"{n}:{ci}:{co}" for n, ci, co in net.layers]
        if list(z["layers"]) != layers:
            raise ValueError(f"{path}: layer table does not match this network")
        net.load_flat(z["params"])
        return net

    # ---------------------------------------------------------------- buffers
    def _buffers(self, shape):
        key = tuple(shape)
        if key in self._bufs:
            return self._bufs[key]
        nz, ny, nx = shape
        if nz % 8 or ny % 8 or nx % 8 or ((nz * ny * nx) // 512) % 16:
            raise ValueError("grid sizes must be multiples of 8 with a coarsest voxel count "
                             "divisible by 16")
        dev = self.p.device
        L = len(LEVELS)
        sh = [(nz >> i, ny >> i, nx >> i) for i in range(L)]
        nv = [a * b * c for a, b, c in sh]

        def bf(nvox, c):
            return torch.zeros((nvox, c), dtype=torch.bfloat16, device=dev)

        b = {"shape": sh, "nv": nv, "x0": bf(nv[0], C_IN)}
        for i in range(L):
            c = LEVELS[i]
            b[f"a{i}"] = bf(nv[i], c)
            b[f"ga{i}"] = bf(nv[i], c)
            b[f"gpre{i}"] = bf(nv[i], c)
            if i > 0:
                b[f"p{i}"] = bf(nv[i], LEVELS[i - 1])
                b[f"gp{i}"] = bf(nv[i], LEVELS[i - 1])
            if i < L - 1:
                b[f"cat{i}"] = bf(nv[i], c + LEVELS[i + 1])
                b[f"gcat{i}"] = bf(nv[i], c + LEVELS[i + 1])
                for k in ("da", "db", "gda", "gdb"):
                    b[f"{k}{i}"] = bf(nv[i], c)
        b["bot"] = bf(nv[L - 1], LEVELS[L - 1])
        b["gbot"] = bf(nv[L - 1], LEVELS[L - 1])
        b["out"] = torch.zeros((self.n_out, nv[0]), dtype=torch.float32, device=dev)
        wsz = max(nn.lbm_nn_wgrad_workspace(sh[self._level(n)], ci, co) for n, ci, co in self.layers)
        b["ws"] = torch.empty(wsz, dtype=torch.uint8, device=dev)
        b["hws"] = torch.empty(nn.lbm_nn_head_workspace(nv[0], self.n_out), dtype=torch.uint8,
                               device=dev)
        self._bufs[key] = b
        return b

    @staticmethod
    def _level(name):
        return int(name[3])

    def _enc_out(self, b, i):
        """View of the output of enc{i}b: the skip part of cat{i}, or the bottom buffer."""
        if i < len(LEVELS) - 1:
            return View(b[f"cat{i}"], 0, LEVELS[i])
        return View(b["bot"])

    def _conv(self, b, name, x, y, relu=True):
        _, ci, co = next(l for l in self.layers if l[0] == name)
        sh = b["shape"][self._level(name)]
        nn.lbm_nn_conv3d(sh, x, ci, self.w_bf(name), self.view(self.p, name + ".b"), y, co,
                         nn.LBM_NN_RELU if relu else 0)

    # ---------------------------------------------------------------- forward
    def forward(self, shape, x0=None):
        """Runs the network on the input in buffer x0 of the grid shape (nz, ny, nx);
        returns the head output, float32 [n_out, nvox] (a buffer reused by later calls)."""
        b = self._buffers(shape)
        if x0 is not None:
            b["x0"].copy_(x0)
        L = len(LEVELS)
        sh = b["shape"]
        h = View(b["x0"])
        for i in range(L):
            if i > 0:
                nn.lbm_nn_pool2(sh[i - 1], LEVELS[i - 1], self._enc_out(b, i - 1), View(b[f"p{i}"]))
                h = View(b[f"p{i}"])
            self._conv(b, f"enc{i}a", h, View(b[f"a{i}"]))
            self._conv(b, f"enc{i}b", View(b[f"a{i}"]), self._enc_out(b, i))
        up = View(b["bot"])
        for i in range(L - 2, -1, -1):
            nn.lbm_nn_up2(sh[i], LEVELS[i + 1], up, View(b[f"cat{i}"], LEVELS[i], LEVELS[i + 1]))
            self._conv(b, f"dec{i}a", View(b[f"cat{i}"]), View(b[f"da{i}"]))
            self._conv(b, f"dec{i}b", View(b[f"da{i}"]), View(b[f"db{i}"]))
            up = View(b[f"db{i}"])
        nn.lbm_nn_head(View(b["db0"]), self.n_out, self.view(self.p, "head.w"),
                       self.view(self.p, "head.b"), out=b["out"])
        return b["out"]

    # ---------------------------------------------------------------- training
    def _conv_bwd(self, b, name, x, y, gy, gx):
        _, ci, co = next(l for l in self.layers if l[0] == name)
        i = self._level(name)
        sh = b["shape"][i]
        gpre = View(b[f"gpre{i}"], 0, co)
        nn.lbm_nn_relu_bwd(co, y, gy, gpre)
        nn.lbm_nn_conv3d_wgrad(sh, x, ci, gpre, co, self.view(self.g, name + ".w"),
                               self.view(self.g, name + ".b"), b["ws"])
        if gx is not None:
            nn.lbm_nn_conv3d(sh, gpre, co, self.wt[name], None, gx, ci, nn.LBM_NN_FLIP)

    def loss_and_grad(self, shape, x0, target, mask, wt, n_mask):
        """Forward, loss and the gradient of every parameter (into self.g)."""
        b = self._buffers(shape)
        self.forward(shape, x0)
        L = len(LEVELS)
        sh = b["shape"]
        loss = nn.lbm_nn_head(View(b["db0"]), self.n_out, self.view(self.p, "head.w"),
                              self.view(self.p, "head.b"), target=target, mask=mask, wt=wt,
                              n_mask=n_mask, gx=View(b["gdb0"]), gwh=self.view(self.g, "head.w"),
                              gbh=self.view(self.g, "head.b"), ws=b["hws"])
        for i in range(L - 1):
            self._conv_bwd(b, f"dec{i}b", View(b[f"da{i}"]), View(b[f"db{i}"]), View(b[f"gdb{i}"]),
                           View(b[f"gda{i}"]))
            self._conv_bwd(b, f"dec{i}a", View(b[f"cat{i}"]), View(b[f"da{i}"]), View(b[f"gda{i}"]),
                           View(b[f"gcat{i}"]))
            g_up = View(b[f"gcat{i}"], LEVELS[i], LEVELS[i + 1])
            nn.lbm_nn_up2_bwd(sh[i], LEVELS[i + 1], g_up,
                              View(b[f"gdb{i + 1}"]) if i + 1 < L - 1 else View(b["gbot"]))
        for i in range(L - 1, -1, -1):
            g_out = View(b[f"gcat{i}"], 0, LEVELS[i]) if i < L - 1 else View(b["gbot"])
            self._conv_bwd(b, f"enc{i}b", View(b[f"a{i}"]), self._enc_out(b, i), g_out,
                           View(b[f"ga{i}"]))
            x_in = View(b[f"p{i}"]) if i > 0 else View(b["x0"])
            self._conv_bwd(b, f"enc{i}a", x_in, View(b[f"a{i}"]), View(b[f"ga{i}"]),
                           View(b[f"gp{i}"]) if i > 0 else None)
            if i > 0:
                # the skip gradient already sits in gcat{i-1}; the pooled path adds to it
                nn.lbm_nn_pool2_bwd(sh[i - 1], LEVELS[i - 1], View(b[f"gp{i}"]),
                                    View(b[f"gcat{i - 1}"], 0, LEVELS[i - 1]), accumulate=True)
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        nn.lbm_nn_adam(self.p, self.g, self.m, self.v, self.pb, lr, beta1, beta2, eps, self.step)
        self._transpose()

    def grads(self):
        """Parameter gradients as host float64 arrays in the oracle's layout."""
        return self._unflatten(self.g)

    def params(self):
        return self._unflatten(self.p)

    def _unflatten(self, flat):
        h = flat.detach().cpu().numpy().astype(np.float64)
        out = {}
        for name, ci, co in self.layers:
            o, k = self.off[name + ".w"]
            out[name + ".w"] = h[o:o + k].reshape(27, co, ci)
            o, k = self.off[name + ".b"]
            out[name + ".b"] = h[o:o + k]
        o, k = self.off["head.w"]
        out["head.w"] = h[o:o + k].reshape(self.n_out, LEVELS[0])
        o, k = self.off["head.b"]
        out["head.b"] = h[o:o + k]
        return out
