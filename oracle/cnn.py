"""Plain CPU reference of the learned-initial-guess network (oracle; test infrastructure).

The network is not in the paper; the paper warm-starts each inner solve from the previous
sweep (paragraph before Alg. 1).  It is a 3-D convolutional encoder-decoder:

* level l has C_l = base * 2^l channels; every convolution is 3x3x3, stride 1, zero padding 1,
  with a bias and a ReLU;
* encoder: level 0 = conv(in -> C_0), conv(C_0 -> C_0); level l >= 1 = 2x2x2 average pooling,
  conv(C_{l-1} -> C_l), conv(C_l -> C_l); the output of each level is kept as a skip tensor;
* decoder, l = L-2 .. 0: nearest-neighbour 2x upsampling of the level-(l+1) output, channel
  concatenation [upsampled, skip_l], conv(C_{l+1} + C_l -> C_l), conv(C_l -> C_l);
* head: 1x1x1 convolution C_0 -> out, no ReLU.

Tensors are channels-last [batch, z, y, x, c]; weights [taps, c_in, c_out] with taps ordered
(dz, dy, dx) in {-1, 0, 1}^3 (z slowest) for 3x3x3 and a single tap for the head.
Everything here is float64 and written with explicit loops over taps (no im2col) so that it
shares nothing with the GPU kernels.  With ``quant=True`` the functions round to bfloat16 at the
points where a BF16 network stores values (weights, hidden activations after bias and ReLU,
pooled activations, and the output gradients fed to the weight- and data-gradient products);
sums are still exact, so the remaining gap to a float32-accumulating implementation is the
accumulation order alone.
"""
from __future__ import annotations

import numpy as np

OFFS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(a):
    """Round to the nearest bfloat16 value, ties to even (via float32), returned as float64.
    The float32 bit pattern u keeps its top 16 bits after adding 0x7fff + (bit 16 of u)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def layer_specs(in_ch, out_ch, base, levels):
    """List of (name, c_in, c_out, taps, relu) in forward order."""
    ch = [base * 2 ** l for l in range(levels)]
    specs = [("enc0a", in_ch, ch[0], 27, True), ("enc0b", ch[0], ch[0], 27, True)]
    for l in range(1, levels):
        specs += [(f"enc{l}a", ch[l - 1], ch[l], 27, True), (f"enc{l}b", ch[l], ch[l], 27, True)]
    for l in range(levels - 2, -1, -1):
        specs += [(f"dec{l}a", ch[l + 1] + ch[l], ch[l], 27, True),
                  (f"dec{l}b", ch[l], ch[l], 27, True)]
    specs.append(("head", ch[0], out_ch, 1, False))
    return specs


def num_params(specs):
    return sum(t * ci * co + co for _, ci, co, t, _ in specs)


def unpack(flat, specs):
    """Flat parameter vector -> list of (W [taps, ci, co], b [co]) in layer order."""
    out, o = [], 0
    for _, ci, co, t, _ in specs:
        W = flat[o:o + t * ci * co].reshape(t, ci, co)
        o += t * ci * co
        b = flat[o:o + co]
        o += co
        out.append((W, b))
    return out


def conv(x, W, b):
    """Zero-padded 3x3x3 (or 1x1x1) convolution, channels-last."""
    taps = W.shape[0]
    n, Z, Y, X, _ = x.shape
    y = np.zeros((n, Z, Y, X, W.shape[2])) + b
    if taps == 1:
        return y + x @ W[0]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    for t, (dz, dy, dx) in enumerate(OFFS):
        y += xp[:, 1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X, :] @ W[t]
    return y


def conv_backward(x, W, gy):
    """Gradients of conv(x, W, b) w.r.t. x, W and b for the upstream gradient gy."""
    taps = W.shape[0]
    n, Z, Y, X, ci = x.shape
    gb = gy.sum(axis=(0, 1, 2, 3))
    if taps == 1:
        return gy @ W[0].T, np.einsum("nzyxi,nzyxo->io", x, gy)[None], gb
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(OFFS):
        sl = (slice(None), slice(1 + dz, 1 + dz + Z), slice(1 + dy, 1 + dy + Y),
              slice(1 + dx, 1 + dx + X), slice(None))
        gW[t] = np.einsum("nzyxi,nzyxo->io", xp[sl], gy)
        gxp[sl] += gy @ W[t].T
    return gxp[:, 1:-1, 1:-1, 1:-1, :], gW, gb


def pool(x):
    n, Z, Y, X, c = x.shape
    return x.reshape(n, Z // 2, 2, Y // 2, 2, X // 2, 2, c).mean(axis=(2, 4, 6))


def pool_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def upsample(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def upsample_backward(g):
    n, Z, Y, X, c = g.shape
    return g.reshape(n, Z // 2, 2, Y // 2, 2, X // 2, 2, c).sum(axis=(2, 4, 6))


def forward(x, flat, in_ch, out_ch, base, levels, keep=False, quant=False):
    specs = layer_specs(in_ch, out_ch, base, levels)
    P = unpack(flat, specs)
    q = bf16 if quant else (lambda a: a)
    acts = {}
    k = 0

    def layer(inp):
        nonlocal k
        W, b = P[k]
        pre = conv(inp, q(W), b)
        out = q(np.maximum(pre, 0.0)) if specs[k][4] else pre
        acts[specs[k][0]] = (inp, out)
        k += 1
        return out

    h = layer(layer(x))
    skips = [h]
    for l in range(1, levels):
        h = layer(layer(q(pool(h))))
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        h = layer(layer(np.concatenate([upsample(h), skips[l]], axis=-1)))
    y = layer(h)
    return (y, acts) if keep else y


def backward(x, flat, gy, in_ch, out_ch, base, levels, quant=False):
    """Parameter gradient (flat, same layout) of <gy, forward(x)>."""
    specs = layer_specs(in_ch, out_ch, base, levels)
    P = unpack(flat, specs)
    q = bf16 if quant else (lambda a: a)
    _, acts = forward(x, flat, in_ch, out_ch, base, levels, keep=True, quant=quant)
    grads = [None] * len(specs)
    k = len(specs) - 1

    def back(g):
        nonlocal k
        name, _, _, _, relu = specs[k]
        inp, out = acts[name]
        if relu:
            g = g * (out > 0)
        gx, gW, _ = conv_backward(inp, q(P[k][0]), q(g))
        grads[k] = (gW, g.sum(axis=(0, 1, 2, 3)))
        k -= 1
        return gx

    ch = [base * 2 ** l for l in range(levels)]
    g = back(gy)                       # head
    gskip = [None] * levels
    for l in range(0, levels - 1):
        g = back(back(g))              # decoder level l (reverse order: l = 0 first)
        gup, gsk = g[..., :ch[l + 1]], g[..., ch[l + 1]:]
        gskip[l] = gsk
        g = upsample_backward(gup)
    for l in range(levels - 1, 0, -1):
        g = back(back(g))              # encoder level l
        g = pool_backward(g)
        g = g + gskip[l - 1]
    back(back(g))                      # encoder level 0
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def init_params(in_ch, out_ch, base, levels, seed):
    """He-normal weights, zero biases (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _, ci, co, t, _ in layer_specs(in_ch, out_ch, base, levels):
        parts.append(rng.normal(size=t * ci * co) * np.sqrt(2.0 / (t * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
