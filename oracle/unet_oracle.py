"""FP64 numpy oracle of the U-Net surrogate (layer definitions, the network's
forward and backward pass, the masked cross-entropy loss and Adam).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the HIP kernels.

The network is not part of the paper: it is the learned warm start that
supplies an initial saturation field to the lattice Boltzmann solver.  Its
layers are textbook operations, written here from their definitions:

  conv3x3   y[n,y,x,o] = b[o] + sum_{ky,kx,i} W[o,ky,kx,i] X[n,y+ky-1,x+kx-1,i]
            (zero outside the grid; cross-correlation, as in deep-learning
            libraries)
  maxpool2  y[n,i,j,c] = max over the 2x2 window at (2i, 2j); the gradient
            goes to the first maximum in raster order
  upconv2   y[n,2i+a,2j+b,o] = b[o] + sum_i W[o,a,b,c] X[n,i,j,c]
  head      z = b + sum_c w[c] X[..., c], s = sigmoid(z)
  loss      mean over masked pixels of  -[t log s + (1-t) log(1-s)]
  adam      Kingma & Ba (2015), Algorithm 1

Layout: NHWC activations, weights [Cout][3][3][Cin] and [Cout][2][2][Cin],
the same as the kernels' interface (an interface, not an implementation).
"""
import numpy as np

LEVELS = (32, 64, 128, 256)
IN_CHANNELS = 8          # 3 input planes, zero-padded to 8 channels


# --------------------------------------------------------------------------
# layers
# --------------------------------------------------------------------------

def conv3x3(x, w, b=None):
    """Zero-padded 3x3 cross-correlation.  x: (N, H, W, Ci), w: (Co, 3, 3, Ci)."""
    n, h, wd, _ = x.shape
    xp = np.zeros((n, h + 2, wd + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((n, h, wd, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + h, kx:kx + wd] @ w[:, ky, kx, :].T
    if b is not None:
        y += b
    return y


def conv3x3_grad(x, w, dy):
    """Gradients of sum(dy * conv3x3(x, w, b)) with respect to x, w and b."""
    n, h, wd, _ = x.shape
    xp = np.zeros((n, h + 2, wd + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            win = xp[:, ky:ky + h, kx:kx + wd]
            dw[:, ky, kx, :] = np.einsum("nyxo,nyxi->oi", dy, win)
            dxp[:, ky:ky + h, kx:kx + wd] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1], dw, dy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def maxpool2(x):
    n, h, wd, c = x.shape
    win = x.reshape(n, h // 2, 2, wd // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, h // 2, wd // 2, 4, c)
    return win.max(axis=3)


def maxpool2_grad(x, dy):
    """Route dy to the first maximum (raster order dy, dx) of each window."""
    n, h, wd, c = x.shape
    win = x.reshape(n, h // 2, 2, wd // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, h // 2, wd // 2, 4, c)
    arg = win.argmax(axis=3)          # numpy takes the first maximum
    sel = np.zeros_like(win)
    np.put_along_axis(sel, arg[:, :, :, None, :], 1.0, axis=3)
    dwin = sel * dy[:, :, :, None, :]
    return dwin.reshape(n, h // 2, wd // 2, 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, h, wd, c)


def upconv2(x, w, b=None):
    """2x2 stride-2 transposed convolution.  w: (Co, 2, 2, Ci)."""
    n, h, wd, _ = x.shape
    y = np.zeros((n, 2 * h, 2 * wd, w.shape[0]))
    for a in range(2):
        for c in range(2):
            y[:, a::2, c::2] = x @ w[:, a, c, :].T
    if b is not None:
        y += b
    return y


def upconv2_grad(x, w, dy):
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for a in range(2):
        for c in range(2):
            g = dy[:, a::2, c::2]
            dx += g @ w[:, a, c, :]
            dw[:, a, c, :] = np.einsum("nyxo,nyxi->oi", g, x)
    return dx, dw, dy.sum(axis=(0, 1, 2))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def head(x, w, b):
    """Logit of the 1x1 head: x (N, H, W, C), w (C,), b scalar."""
    return x @ w + b


def masked_bce(z, t, mask):
    """Mean binary cross-entropy of sigmoid(z) against t over mask != 0."""
    s = sigmoid(z)
    m = mask.astype(bool)
    return float(-(t[m] * np.log(s[m]) + (1 - t[m]) * np.log(1 - s[m])).sum() / m.sum())


def masked_bce_grad(z, t, mask):
    """d loss / d z."""
    m = mask.astype(bool)
    return np.where(m, sigmoid(z) - t, 0.0) / m.sum()


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    """One Adam update (returns new p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------

def layer_specs(levels=LEVELS, cin=IN_CHANNELS):
    """(name, kind, cin, cout) in forward order; kind 'conv' (3x3 + ReLU) or
    'up' (2x2 transposed, no activation); the head is separate."""
    c = list(levels)
    specs = []
    prev = cin
    for k, ch in enumerate(c):
        specs += [(f"enc{k}a", "conv", prev, ch), (f"enc{k}b", "conv", ch, ch)]
        prev = ch
    for k in range(len(c) - 2, -1, -1):
        specs += [(f"up{k}", "up", c[k + 1], c[k]),
                  (f"dec{k}a", "conv", 2 * c[k], c[k]), (f"dec{k}b", "conv", c[k], c[k])]
    return specs


def init_params(seed=0, levels=LEVELS, cin=IN_CHANNELS):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, kind, ci, co in layer_specs(levels, cin):
        taps = 3 if kind == "conv" else 2
        p[name + ".w"] = rng.normal(0, np.sqrt(2.0 / (taps * taps * ci)), (co, taps, taps, ci))
        p[name + ".b"] = np.zeros(co)
    p["head.w"] = rng.normal(0, np.sqrt(1.0 / levels[0]), levels[0])
    p["head.b"] = np.zeros(1)
    return p


def forward(p, x, levels=LEVELS):
    """x: (N, H, W, IN_CHANNELS).  Returns (logit (N, H, W), cache)."""
    L = len(levels)
    a = {}
    h = x
    skips = []
    for k in range(L):
        a[f"in_enc{k}a"] = h
        h = relu(conv3x3(h, p[f"enc{k}a.w"], p[f"enc{k}a.b"]))
        a[f"enc{k}a"] = h
        h = relu(conv3x3(h, p[f"enc{k}b.w"], p[f"enc{k}b.b"]))
        a[f"enc{k}b"] = h
        if k < L - 1:
            skips.append(h)
            h = maxpool2(h)
    for k in range(L - 2, -1, -1):
        a[f"in_up{k}"] = h
        u = upconv2(h, p[f"up{k}.w"], p[f"up{k}.b"])
        cat = np.concatenate([skips[k], u], axis=3)   # skip first, then upsampled
        a[f"cat{k}"] = cat
        h = relu(conv3x3(cat, p[f"dec{k}a.w"], p[f"dec{k}a.b"]))
        a[f"dec{k}a"] = h
        h = relu(conv3x3(h, p[f"dec{k}b.w"], p[f"dec{k}b.b"]))
        a[f"dec{k}b"] = h
    z = head(h, p["head.w"], p["head.b"][0])
    a["top"] = h
    return z, a


def backward(p, a, dz, levels=LEVELS):
    """Gradients of sum(dz * logit) for every parameter."""
    L = len(levels)
    g = {}
    top = a["top"]
    g["head.w"] = np.einsum("nyx,nyxc->c", dz, top)
    g["head.b"] = np.array([dz.sum()])
    dh = dz[..., None] * p["head.w"]
    dskip = [None] * (L - 1)
    for k in range(0, L - 1):
        # decoder levels in reverse forward order: full resolution (k = 0) first
        dh = dh * (a[f"dec{k}b"] > 0)
        dx, g[f"dec{k}b.w"], g[f"dec{k}b.b"] = conv3x3_grad(a[f"dec{k}a"], p[f"dec{k}b.w"], dh)
        dh = dx * (a[f"dec{k}a"] > 0)
        dcat, g[f"dec{k}a.w"], g[f"dec{k}a.b"] = conv3x3_grad(a[f"cat{k}"], p[f"dec{k}a.w"], dh)
        c = levels[k]
        dskip[k] = dcat[..., :c]
        du = dcat[..., c:]
        dh, g[f"up{k}.w"], g[f"up{k}.b"] = upconv2_grad(a[f"in_up{k}"], p[f"up{k}.w"], du)
    # dh is now the gradient at the bottleneck output enc{L-1}b
    for k in range(L - 1, -1, -1):
        if k < L - 1:
            dh = dskip[k] + maxpool2_grad(a[f"enc{k}b"], dh)
        dh = dh * (a[f"enc{k}b"] > 0)
        dx, g[f"enc{k}b.w"], g[f"enc{k}b.b"] = conv3x3_grad(a[f"enc{k}a"], p[f"enc{k}b.w"], dh)
        dh = dx * (a[f"enc{k}a"] > 0)
        dh, g[f"enc{k}a.w"], g[f"enc{k}a.b"] = conv3x3_grad(a[f"in_enc{k}a"], p[f"enc{k}a.w"], dh)
    return g
