"""U-Net surrogate of the steady saturation field, trained and run on the
library's own BF16-MFMA kernels (include/unet.h), and the warm start it gives
the lattice Boltzmann solver.

The network: four levels of two (3x3 conv -> ReLU) at 32/64/128/256 channels,
2x2 max pooling down, 2x2 transposed convolutions up, skip concatenation
(encoder features first, upsampled second), and a 1x1 head with a sigmoid.
Input: three planes (solid mask, contact-angle plane, pressure-step plane)
zero-padded to 8 channels, NHWC BF16.  Output: the per-node fraction of the
non-wetting component, rho1 / (rho1 + rho2).  FP32 master weights and Adam
moments, BF16 weights and activations in the kernels, FP32 accumulation.

This module only marshals arguments and owns device buffers (torch tensors);
every layer runs in the library's kernels.  There is no fallback path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lbm as _lbm

LEVELS = (32, 64, 128, 256)
IN_CH = 8

_ready = False


def lib():
    """liblbm.so with the unet_* prototypes set."""
    global _ready
    L = _lbm.lib()
    if not _ready:
        vp, i32, i64, f32 = C.c_void_p, C.c_int, C.c_int64, C.c_float
        sig = {
            "unet_mfma_probe": [vp, vp, vp, vp],
            "unet_conv3x3_fwd": [vp, i32, i32, i32, i32, i32, i32, vp, vp, i32, vp, i32, i32, i32, vp],
            "unet_conv3x3_flip": [vp, i32, i32, vp, vp],
            "unet_conv3x3_wgrad": [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, i32, vp, vp, vp, i32, vp],
            "unet_conv3x3_wgrad_noalloc": [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, i32, vp, vp, i32, vp],
            "unet_relu_bwd": [vp, i32, i32, i32, i32, vp, i32, i32, vp],
            "unet_maxpool_fwd": [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, vp],
            "unet_maxpool_bwd": [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, vp, i32, i32, i32, vp],
            "unet_upconv_fwd": [vp, i32, i32, i32, i32, i32, i32, vp, vp, i32, vp, i32, i32, vp],
            "unet_upconv_bwd_data": [vp, i32, i32, i32, i32, i32, i32, vp, i32, vp, vp, i32, i32, vp],
            "unet_upconv_wgrad": [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, i32, vp, vp, vp, vp],
            "unet_head_fwd": [vp, i32, i32, i32, vp, vp, vp, vp],
            "unet_head_loss_bwd": [vp, i32, i32, i32, vp, vp, vp, vp, f32, vp, vp, vp, vp, vp, vp],
            "unet_adam": [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp],
            "unet_to_bf16": [vp, vp, i64, vp],
            "unet_to_f32": [vp, vp, i64, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        for name in ("unet_wgrad_scratch_floats", "unet_head_scratch_floats"):
            getattr(L, name).restype = C.c_int64
        L.unet_wgrad_scratch_floats.argtypes = [i32, i32, i32, i32, i32, i32]
        L.unet_head_scratch_floats.argtypes = [i32, i32]
        _ready = True
    return L


EXPORTS = [
    "unet_mfma_probe", "unet_conv3x3_fwd", "unet_conv3x3_flip", "unet_wgrad_scratch_floats",
    "unet_conv3x3_wgrad", "unet_conv3x3_wgrad_noalloc", "unet_relu_bwd", "unet_maxpool_fwd", "unet_maxpool_bwd", "unet_upconv_fwd",
    "unet_upconv_bwd_data", "unet_upconv_wgrad", "unet_head_fwd", "unet_head_scratch_floats",
    "unet_head_loss_bwd", "unet_adam", "unet_to_bf16", "unet_to_f32",
]


def call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise RuntimeError(f"{name} failed with status {st}")


def ptr(t, offset=0):
    """Device address of element `offset` of a torch tensor."""
    return t.data_ptr() + offset * t.element_size()


def layer_specs(levels=LEVELS, cin=IN_CH):
    """(name, kind, cin, cout) in forward order."""
    specs = []
    prev = cin
    for k, ch in enumerate(levels):
        specs += [(f"enc{k}a", "conv", prev, ch), (f"enc{k}b", "conv", ch, ch)]
        prev = ch
    for k in range(len(levels) - 2, -1, -1):
        specs += [(f"up{k}", "up", levels[k + 1], levels[k]),
                  (f"dec{k}a", "conv", 2 * levels[k], levels[k]),
                  (f"dec{k}b", "conv", levels[k], levels[k])]
    return specs


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """float -> BF16 bit patterns, round to nearest even (host-side input prep)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_to_float(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


class UNet:
    """Weights, optimiser state and activation buffers on one device."""

    def __init__(self, levels=LEVELS, seed=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.levels = tuple(levels)
        self.L = len(self.levels)
        self.device = torch.device(device)
        self.specs = layer_specs(self.levels)
        # flat parameter vector; every tensor starts on a 64-element boundary
        self.off = {}
        pos = 0

        def take(name, count):
            nonlocal pos
            self.off[name] = (pos, count)
            pos += (count + 63) // 64 * 64

        self.shapes = {}
        for name, kind, ci, co in self.specs:
            t = 3 if kind == "conv" else 2
            self.shapes[name + ".w"] = (co, t, t, ci)
            self.shapes[name + ".b"] = (co,)
        self.shapes["head.w"] = (self.levels[0],)
        self.shapes["head.b"] = (1,)
        for name, shp in self.shapes.items():
            take(name, int(np.prod(shp)))
        self.n_params = pos
        f32 = torch.float32
        self.p = torch.zeros(pos, dtype=f32, device=self.device)
        self.pb = torch.zeros(pos, dtype=torch.int16, device=self.device)
        self.g = torch.zeros(pos, dtype=f32, device=self.device)
        self.m = torch.zeros(pos, dtype=f32, device=self.device)
        self.v = torch.zeros(pos, dtype=f32, device=self.device)
        self.adam_t = 0
        rng = np.random.default_rng(seed)
        init = {}
        for name, kind, ci, co in self.specs:
            t = 3 if kind == "conv" else 2
            init[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (t * t * ci)), (co, t, t, ci))
            init[name + ".b"] = np.zeros(co)
        init["head.w"] = rng.normal(0.0, np.sqrt(1.0 / self.levels[0]), self.levels[0])
        init["head.b"] = np.zeros(1)
        self.set_params(init)
        self._shape = None

    # ---------------------------------------------------------------- params
    def stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def set_params(self, params: dict):
        host = np.zeros(self.n_params, np.float32)
        for name, (o, n) in self.off.items():
            a = np.asarray(params[name], dtype=np.float64)
            assert a.shape == self.shapes[name], (name, a.shape)
            host[o:o + n] = a.ravel()
        self.p.copy_(self.torch.from_numpy(host))
        call("unet_to_bf16", ptr(self.p), ptr(self.pb), self.n_params, self.stream())

    def get_params(self) -> dict:
        host = self.p.cpu().numpy()
        return {k: host[o:o + n].reshape(self.shapes[k]).copy() for k, (o, n) in self.off.items()}

    def get_grads(self) -> dict:
        host = self.g.cpu().numpy()
        return {k: host[o:o + n].reshape(self.shapes[k]).copy() for k, (o, n) in self.off.items()}

    def save(self, path):
        """Weights as the kernels use them: BF16 bit patterns for the
        convolution weights, FP32 for biases and the head."""
        params = self.get_params()
        bits = self.pb.cpu().numpy().view(np.uint16)
        out = {}
        for k, v in params.items():
            if k.endswith(".w") and not k.startswith("head"):
                o, n = self.off[k]
                out[k] = bits[o:o + n].reshape(self.shapes[k]).copy()
            else:
                out[k] = v.astype(np.float32)
        np.savez(path, levels=np.array(self.levels), **out)

    @classmethod
    def load(cls, path, device="cuda:0"):
        with np.load(path, allow_pickle=False) as z:
            net = cls(levels=tuple(int(v) for v in z["levels"]), device=device)
            params = {}
            for k in net.shapes:
                a = z[k]
                params[k] = bf16_to_float(a) if a.dtype == np.uint16 else a
            net.set_params(params)
        return net

    def _w(self, name):        # BF16 weight address
        return ptr(self.pb, self.off[name + ".w"][0])

    def _p32(self, name):      # FP32 master address
        return ptr(self.p, self.off[name][0])

    def _g(self, name):
        return ptr(self.g, self.off[name][0])

    # --------------------------------------------------------------- buffers
    def _buffers(self, n, h, w):
        if self._shape == (n, h, w):
            return
        torch = self.torch
        assert h % (1 << (self.L - 1)) == 0 and w % (1 << (self.L - 1)) == 0
        bf = lambda *s: torch.zeros(s, dtype=torch.int16, device=self.device)  # noqa: E731
        c = self.levels
        hs = [(h >> k, w >> k) for k in range(self.L)]
        self.hs = hs
        A = {}
        A["x"] = bf(n, h, w, IN_CH)
        for k in range(self.L):
            hk, wk = hs[k]
            A[f"enc{k}a"] = bf(n, hk, wk, c[k])
            if k < self.L - 1:
                A[f"cat{k}"] = bf(n, hk, wk, 2 * c[k])        # [enc{k}b | up{k}]
                A[f"pool{k}"] = bf(n, hk // 2, wk // 2, c[k])
                A[f"dec{k}a"] = bf(n, hk, wk, c[k])
                A[f"dec{k}b"] = bf(n, hk, wk, c[k])
            else:
                A[f"enc{k}b"] = bf(n, hk, wk, c[k])
        G = {}
        for k in range(self.L):
            hk, wk = hs[k]
            G[f"enc{k}a"] = bf(n, hk, wk, c[k])
            if k < self.L - 1:
                G[f"cat{k}"] = bf(n, hk, wk, 2 * c[k])
                G[f"dec{k}a"] = bf(n, hk, wk, c[k])
                G[f"dec{k}b"] = bf(n, hk, wk, c[k])
                G[f"pool{k}"] = bf(n, hk // 2, wk // 2, c[k])
            else:
                G[f"enc{k}b"] = bf(n, hk, wk, c[k])
        self.A, self.G = A, G
        maxw = max(co * 9 * ci for _, _, ci, co in self.specs)
        self.wt = bf(maxw)
        L = lib()
        part = 0
        for k in range(self.L):
            hk, wk = hs[k]
            for ci, co, taps, hh, ww in ((c[k], c[k], 9, hk, wk), (IN_CH if k == 0 else c[k - 1], c[k], 9, hk, wk),
                                         (2 * c[k], c[k], 9, hk, wk)):
                part = max(part, L.unet_wgrad_scratch_floats(n, hh, ww, ci, co, taps))
            if k < self.L - 1:
                part = max(part, L.unet_wgrad_scratch_floats(n, hs[k + 1][0], hs[k + 1][1], c[k + 1], c[k], 4))
        self.partial = torch.zeros(part, dtype=torch.float32, device=self.device)
        self.head_scratch = torch.zeros(L.unet_head_scratch_floats(n * h * w, c[0]), dtype=torch.float32,
                                        device=self.device)
        self.sat = torch.zeros((n, h, w), dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._shape = (n, h, w)

    # --------------------------------------------------------------- forward
    def _conv(self, x, x_cs, x_co, n, h, w, cin, name, cout, y, y_cs, y_co, relu=1):
        call("unet_conv3x3_fwd", ptr(x), n, h, w, cin, x_cs, x_co, self._w(name), self._p32(name + ".b"),
             cout, ptr(y), y_cs, y_co, relu, self.stream())

    def forward(self, x_bits):
        """x_bits: int16 tensor (n, h, w, 8) of BF16 bit patterns on the device.
        Returns the saturation prediction (n, h, w) FP32 (a view of an internal
        buffer, valid until the next forward)."""
        n, h, w, ch = x_bits.shape
        assert ch == IN_CH
        self._buffers(n, h, w)
        A, c, s = self.A, self.levels, self.stream()
        A["x"].copy_(x_bits)
        inp, in_c = A["x"], IN_CH
        for k in range(self.L):
            hk, wk = self.hs[k]
            self._conv(inp, in_c, 0, n, hk, wk, in_c, f"enc{k}a", c[k], A[f"enc{k}a"], c[k], 0)
            if k < self.L - 1:
                self._conv(A[f"enc{k}a"], c[k], 0, n, hk, wk, c[k], f"enc{k}b", c[k], A[f"cat{k}"], 2 * c[k], 0)
                call("unet_maxpool_fwd", ptr(A[f"cat{k}"]), n, hk, wk, c[k], 2 * c[k], 0, ptr(A[f"pool{k}"]),
                     c[k], 0, s)
                inp, in_c = A[f"pool{k}"], c[k]
            else:
                self._conv(A[f"enc{k}a"], c[k], 0, n, hk, wk, c[k], f"enc{k}b", c[k], A[f"enc{k}b"], c[k], 0)
        below, below_c = A[f"enc{self.L - 1}b"], c[self.L - 1]
        for k in range(self.L - 2, -1, -1):
            hk, wk = self.hs[k]
            h1, w1 = self.hs[k + 1]
            call("unet_upconv_fwd", ptr(below), n, h1, w1, below_c, below_c, 0, self._w(f"up{k}"),
                 self._p32(f"up{k}.b"), c[k], ptr(A[f"cat{k}"]), 2 * c[k], c[k], s)
            self._conv(A[f"cat{k}"], 2 * c[k], 0, n, hk, wk, 2 * c[k], f"dec{k}a", c[k], A[f"dec{k}a"], c[k], 0)
            self._conv(A[f"dec{k}a"], c[k], 0, n, hk, wk, c[k], f"dec{k}b", c[k], A[f"dec{k}b"], c[k], 0)
            below, below_c = A[f"dec{k}b"], c[k]
        call("unet_head_fwd", ptr(A["dec0b"]), n * h * w, c[0], c[0], self._p32("head.w"), self._p32("head.b"),
             ptr(self.sat), s)
        return self.sat

    # -------------------------------------------------------------- backward
    def backward(self, target, mask, count=None):
        """Masked binary cross-entropy of the last forward against `target`
        (n, h, w) FP32 over `mask` (n, h, w) uint8 with `count` nonzero
        entries; fills the gradients and returns the loss as a 1-element
        device tensor."""
        n, h, w = self._shape
        A, G, c, s = self.A, self.G, self.levels, self.stream()
        if count is None:
            count = int(mask.sum().item())
        scale = 1.0 / max(count, 1)
        call("unet_head_loss_bwd", ptr(A["dec0b"]), n * h * w, c[0], c[0], self._p32("head.w"),
             self._p32("head.b"), ptr(target), ptr(mask), scale, ptr(self.loss), ptr(G["dec0b"]),
             self._g("head.w"), self._g("head.b"), ptr(self.head_scratch), s)
        wt, part = self.wt, self.partial

        def conv_back(x, x_cs, x_co, y, y_cs, y_co, gy, gy_cs, gy_co, hh, ww, cin, cout, name, gx, gx_cs, gx_co):
            """Through act(conv(x)) = y: mask gy by ReLU, weight/bias grads,
            and (if gx is given) the data gradient into gx."""
            call("unet_relu_bwd", ptr(y), n * hh * ww, cout, y_cs, y_co, ptr(gy), gy_cs, gy_co, s)
            call("unet_conv3x3_wgrad", ptr(x), n, hh, ww, cin, x_cs, x_co, ptr(gy), cout, gy_cs, gy_co,
                 self._g(name + ".w"), self._g(name + ".b"), ptr(part), 0, s)
            if gx is not None:
                call("unet_conv3x3_flip", self._w(name), cout, cin, ptr(wt), s)
                call("unet_conv3x3_fwd", ptr(gy), n, hh, ww, cout, gy_cs, gy_co, ptr(wt), None, cin, ptr(gx),
                     gx_cs, gx_co, 0, s)

        for k in range(self.L - 1):
            hk, wk = self.hs[k]
            h1, w1 = self.hs[k + 1]
            conv_back(A[f"dec{k}a"], c[k], 0, A[f"dec{k}b"], c[k], 0, G[f"dec{k}b"], c[k], 0, hk, wk, c[k], c[k],
                      f"dec{k}b", G[f"dec{k}a"], c[k], 0)
            conv_back(A[f"cat{k}"], 2 * c[k], 0, A[f"dec{k}a"], c[k], 0, G[f"dec{k}a"], c[k], 0, hk, wk, 2 * c[k],
                      c[k], f"dec{k}a", G[f"cat{k}"], 2 * c[k], 0)
            below = A[f"dec{k + 1}b"] if k + 1 < self.L - 1 else A[f"enc{self.L - 1}b"]
            gbelow = G[f"dec{k + 1}b"] if k + 1 < self.L - 1 else G[f"enc{self.L - 1}b"]
            call("unet_upconv_wgrad", ptr(below), n, h1, w1, c[k + 1], c[k + 1], 0, ptr(G[f"cat{k}"]), c[k],
                 2 * c[k], c[k], self._g(f"up{k}.w"), self._g(f"up{k}.b"), ptr(part), s)
            call("unet_upconv_bwd_data", ptr(G[f"cat{k}"]), n, h1, w1, c[k], 2 * c[k], c[k], self._w(f"up{k}"),
                 c[k + 1], ptr(wt), ptr(gbelow), c[k + 1], 0, s)
        for k in range(self.L - 1, -1, -1):
            hk, wk = self.hs[k]
            if k < self.L - 1:
                yb, yb_cs, gyb, gyb_cs = A[f"cat{k}"], 2 * c[k], G[f"cat{k}"], 2 * c[k]
                call("unet_maxpool_bwd", ptr(A[f"cat{k}"]), n, hk, wk, c[k], 2 * c[k], 0, ptr(G[f"pool{k}"]),
                     c[k], 0, ptr(G[f"cat{k}"]), 2 * c[k], 0, 1, s)
            else:
                yb, yb_cs, gyb, gyb_cs = A[f"enc{k}b"], c[k], G[f"enc{k}b"], c[k]
            conv_back(A[f"enc{k}a"], c[k], 0, yb, yb_cs, 0, gyb, gyb_cs, 0, hk, wk, c[k], c[k], f"enc{k}b",
                      G[f"enc{k}a"], c[k], 0)
            if k > 0:
                x, x_c = A[f"pool{k - 1}"], c[k - 1]
                conv_back(x, x_c, 0, A[f"enc{k}a"], c[k], 0, G[f"enc{k}a"], c[k], 0, hk, wk, x_c, c[k],
                          f"enc{k}a", G[f"pool{k - 1}"], x_c, 0)
            else:
                conv_back(A["x"], IN_CH, 0, A["enc0a"], c[0], 0, G["enc0a"], c[0], 0, hk, wk, IN_CH, c[0],
                          "enc0a", None, 0, 0)
        return self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.adam_t += 1
        call("unet_adam", ptr(self.p), ptr(self.g), ptr(self.m), ptr(self.v), ptr(self.pb), self.n_params,
             lr, beta1, beta2, eps, self.adam_t, self.stream())

    def train_step(self, x_bits, target, mask, lr=1e-3, count=None):
        self.forward(x_bits)
        loss = self.backward(target, mask, count)
        self.adam(lr)
        return loss

    def flops_per_image(self, h, w):
        """Multiply-adds x 2 of the convolutions in one forward pass."""
        f = 0
        for name, kind, ci, co in self.specs:
            lvl = int(name[3]) if name.startswith(("enc", "dec")) else int(name[2:])
            hh, ww = h >> lvl, w >> lvl
            if kind == "conv":
                f += 2 * hh * ww * 9 * ci * co
            else:  # one tap per output pixel
                f += 2 * hh * ww * ci * co
        return f + 2 * h * w * self.levels[0]


# ------------------------------------------------------------------ problem I/O
THETA_MID, THETA_HALF = 90.0, 60.0          # contact-angle plane: (theta - 90) / 60
LOGDP_MID, LOGDP_HALF = -3.15, 0.85         # pressure plane: (log10 dp + 3.15) / 0.85


def features(mask: np.ndarray, theta: float, dp: float) -> np.ndarray:
    """Network input (h, w, 8) float: solid mask, contact-angle plane,
    pressure-step plane, five zero channels."""
    h, w = mask.shape
    x = np.zeros((h, w, IN_CH), np.float32)
    x[..., 0] = mask
    x[..., 1] = (theta - THETA_MID) / THETA_HALF
    x[..., 2] = (np.log10(dp) - LOGDP_MID) / LOGDP_HALF
    return x


def saturation_field(rho: np.ndarray) -> np.ndarray:
    """Per-node non-wetting fraction rho1 / (rho1 + rho2) (0 at solid nodes)."""
    tot = rho[0] + rho[1]
    return np.where(tot > 0, rho[0] / np.where(tot > 0, tot, 1.0), 0.0)


def warm_start_density(problem, sat: np.ndarray, threshold: float = 0.5) -> np.ndarray:
    """Initial densities from a predicted saturation field: inside the porous
    window a fluid node is non-wetting-rich (rho1, rho2) = (major, minor)
    where the prediction exceeds `threshold`, wetting-rich otherwise; the
    reservoirs keep the cold-start state."""
    rho = np.array(problem.rho0, dtype=np.float64, copy=True)
    fluid = problem.mask == 0
    major = float(rho[1][fluid].max())
    minor = float(rho[0][fluid].min())
    win = np.zeros_like(fluid)
    win[:, problem.porous_x0:problem.porous_x1] = True
    sel = fluid & win
    nw = sel & (sat > threshold)
    w = sel & ~(sat > threshold)
    rho[0][nw], rho[1][nw] = major, minor
    rho[0][w], rho[1][w] = minor, major
    return rho


def full_saturation(problem, sat: np.ndarray) -> np.ndarray:
    """A saturation field over the whole grid for the solver's warm start
    (lbm_init_from_saturation): the prediction inside the porous window, the
    cold start's phases (1 where component 1 is the majority) outside it, 0
    at solid nodes.  With the threshold 0.5 it sets the same densities as
    warm_start_density."""
    rho = np.asarray(problem.rho0)
    out = (rho[0] > rho[1]).astype(np.float32)
    win = np.zeros(problem.mask.shape, dtype=bool)
    win[:, problem.porous_x0:problem.porous_x1] = True
    out[win] = np.asarray(sat, dtype=np.float32)[win]
    out[problem.mask != 0] = 0.0
    return out


def predict(net: "UNet", problems, batch: int = 8) -> np.ndarray:
    """Saturation predictions (k, h, w) for problems with attributes theta, dp."""
    import torch
    out = []
    for i in range(0, len(problems), batch):
        chunk = problems[i:i + batch]
        x = np.stack([features(p.mask, p.theta, p.dp) for p in chunk])
        xb = torch.from_numpy(bf16_bits(x).view(np.int16)).to(net.device)
        out.append(net.forward(xb).cpu().numpy().copy())
    return np.concatenate(out)
