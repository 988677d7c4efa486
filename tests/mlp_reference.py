"""FP64 numpy forward/backward of the MLP the library trains (test
infrastructure).  Layout of the flat parameter vector: per layer W [out][in]
then b [out]; SiLU between layers, linear output, mean squared error."""
import numpy as np


def shapes(d_in, width, n_layers):
    out = []
    for l in range(n_layers):
        i = d_in if l == 0 else width
        o = 1 if l == n_layers - 1 else width
        out.append((o, i))
    return out


def unpack(p, d_in, width, n_layers):
    layers, off = [], 0
    for o, i in shapes(d_in, width, n_layers):
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        layers.append((W, b))
    return layers


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(p, X, d_in, width, n_layers):
    A = X.astype(np.float64)
    cache = []
    for l, (W, b) in enumerate(unpack(p.astype(np.float64), d_in, width,
                                      n_layers)):
        Z = A @ W.T + b
        cache.append((A, Z))
        A = Z * _sig(Z) if l < n_layers - 1 else Z
    return A[:, 0], cache


def loss_and_grad(p, X, t, d_in, width, n_layers):
    y, cache = forward(p, X, d_in, width, n_layers)
    B = X.shape[0]
    loss = np.mean((y - t) ** 2)
    dZ = (2.0 * (y - t) / B)[:, None]
    grads = []
    layers = unpack(p.astype(np.float64), d_in, width, n_layers)
    for l in range(n_layers - 1, -1, -1):
        A_in, Z = cache[l]
        W, b = layers[l]
        grads.append((dZ.T @ A_in, dZ.sum(axis=0)))
        if l == 0:
            break
        dA = dZ @ W
        Zp = cache[l - 1][1]
        s = _sig(Zp)
        dZ = dA * s * (1.0 + Zp * (1.0 - s))
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db.ravel())
    return loss, np.concatenate(flat)
