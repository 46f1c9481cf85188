"""Residual CNN surrogate of the GLR prior step (oracle; test infrastructure).

The network f maps a 2-channel slice (the pre-prior image x and a constant
map of the noise level sigma_t) to a residual, and the surrogate estimate is
x + f(x, sigma).  f is five 3x3 convolutions with zero padding (channels
2 -> 64 -> 64 -> 64 -> 64 -> 1) with ReLU after the first four.  A
convolution is a cross-correlation:
    out[o, y, x] = b[o] + sum_c sum_{dy, dx in 0..2} W[o, c, dy, dx] * in[c, y + dy - 1, x + dx - 1].

Parameters are kept as one flat FP64/FP32 vector in the order
W1 [64][2][3][3], b1 [64], W2, b2, W3, b3, W4, b4, W5 [1][64][3][3], b5 [1].

``bf16=True`` mirrors the precision of the GPU network: weights, the network
input and every hidden activation are rounded to BF16 (round to nearest
even) before they enter a convolution, and so are the back-propagated
pre-activation gradients of layers 1-4 before they enter the data and weight
gradient products; everything else is exact FP64.  The loss is the mean
squared error over all pixels.

Plain slow code: every step is written out; no fusion.
"""
import numpy as np

CH = 64          # hidden channels of the network (tests also use smaller ones)


def layers(ch=CH):
    return [(2, ch), (ch, ch), (ch, ch), (ch, ch), (ch, 1)]


def param_shapes(ch=CH):
    out = []
    for ci, co in layers(ch):
        out.append((co, ci, 3, 3))
        out.append((co,))
    return out


def param_count(ch=CH):
    return int(sum(np.prod(s) for s in param_shapes(ch)))


def unflatten(theta, ch=CH):
    theta = np.asarray(theta, dtype=np.float64)
    ps, o = [], 0
    for s in param_shapes(ch):
        n = int(np.prod(s))
        ps.append(theta[o:o + n].reshape(s))
        o += n
    assert o == theta.size
    return ps


def flatten(ps):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in ps])


def bf16_round(a):
    """Round float values to the nearest BF16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, W, b):
    """x [B][Ci][h][w], W [Co][Ci][3][3], b [Co] -> [B][Co][h][w]."""
    B, Ci, h, w = x.shape
    xp = np.zeros((B, Ci, h + 2, w + 2))
    xp[:, :, 1:h + 1, 1:w + 1] = x
    out = np.broadcast_to(np.asarray(b, np.float64)[None, :, None, None],
                          (B, W.shape[0], h, w)).copy()
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("bchw,oc->bohw", xp[:, :, dy:dy + h, dx:dx + w], W[:, :, dy, dx])
    return out


def conv3x3_data_grad(g, W, shape_in):
    """Gradient of sum(g * conv3x3(x, W, 0)) with respect to x."""
    B, Ci, h, w = shape_in
    gx = np.zeros((B, Ci, h + 2, w + 2))
    for dy in range(3):
        for dx in range(3):
            gx[:, :, dy:dy + h, dx:dx + w] += np.einsum("bohw,oc->bchw", g, W[:, :, dy, dx])
    return gx[:, :, 1:h + 1, 1:w + 1]


def conv3x3_weight_grad(g, x):
    """Gradient of sum(g * conv3x3(x, W, b)) with respect to W and b."""
    B, Ci, h, w = x.shape
    xp = np.zeros((B, Ci, h + 2, w + 2))
    xp[:, :, 1:h + 1, 1:w + 1] = x
    gW = np.zeros((g.shape[1], Ci, 3, 3))
    for dy in range(3):
        for dx in range(3):
            gW[:, :, dy, dx] = np.einsum("bohw,bchw->oc", g, xp[:, :, dy:dy + h, dx:dx + w])
    return gW, g.sum(axis=(0, 2, 3))


def network_input(x, sigma):
    """x [B][h][w], sigma [B] -> [B][2][h][w] (image, constant sigma map)."""
    x = np.asarray(x, np.float64)
    s = np.broadcast_to(np.asarray(sigma, np.float64)[:, None, None], x.shape)
    return np.stack([x, s], axis=1)


def forward(theta, x, sigma, bf16=False, keep=False, ch=CH):
    """Surrogate estimate x + f(x, sigma) for slices x [B][h][w]."""
    ps = unflatten(theta, ch)
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    a = rnd(network_input(x, sigma))
    acts = [a]
    for layer in range(5):
        W, b = rnd(ps[2 * layer]), ps[2 * layer + 1]
        z = conv3x3(a, W, b)
        if layer < 4:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
    out = np.asarray(x, np.float64) + z[:, 0]
    return (out, acts) if keep else out


def loss_and_grad(theta, x, sigma, target, bf16=False, ch=CH):
    """MSE loss mean((x + f - target)^2) and its gradient (flat, FP64)."""
    ps = unflatten(theta, ch)
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    out, acts = forward(theta, x, sigma, bf16=bf16, keep=True, ch=ch)
    n = out.size
    r = out - np.asarray(target, np.float64)
    loss = float(np.sum(r * r) / n)
    g = (2.0 / n) * r[:, None]                  # d loss / d z5   [B][1][h][w]
    grads = [None] * 10
    for layer in range(4, -1, -1):
        W = rnd(ps[2 * layer])
        a_in = acts[layer]
        gW, gb = conv3x3_weight_grad(g, a_in)
        grads[2 * layer], grads[2 * layer + 1] = gW, gb
        if layer > 0:
            ga = conv3x3_data_grad(g, W, a_in.shape)
            g = rnd(ga * (a_in > 0))             # through the ReLU of the layer below
    return loss, flatten(grads)


def adam_step(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def judge_deviation(x_cnn, x_glr, covered):
    """Relative deviation of the surrogate from the subset GLR estimate on the
    covered pixels: ||(x_cnn - x_glr)|_cov|| / ||x_glr|_cov||; +inf when the
    surrogate is not finite anywhere or nothing is covered."""
    c = np.asarray(covered, bool)
    a = np.asarray(x_cnn)[..., c] if c.shape != np.shape(x_cnn) else np.asarray(x_cnn)[c]
    b = np.asarray(x_glr)[..., c] if c.shape != np.shape(x_glr) else np.asarray(x_glr)[c]
    if not np.all(np.isfinite(a)):
        return float("inf")
    den = float(np.sqrt(np.sum(np.abs(b) ** 2)))
    if den == 0.0:
        return float("inf")
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2)) / den)
