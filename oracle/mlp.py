"""Oracle of the learned parameter selector (test infrastructure only).

Plain float64 numpy definitions of the selector network, its loss, the gradient of the loss by
back-propagation written layer by layer, and one Adam step.  The thesis leaves the choice of
DKSS parameters open beyond its asymptotic rule (Sec. 4.1; its outlook, Chapter 5); the network
here is the library's own addition and is defined by its interface:

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3
    loss = sum_n sum_k mask[n,k] (y[n,k] - t[n,k])^2 / mask_sum

Parameters are one flat vector in the order W1[HID][IN], b1[HID], W2[HID][HID], b2[HID],
W3[OUT][HID], b3[OUT] (row-major; row = output unit).  Adam: Kingma and Ba, "Adam: A Method for
Stochastic Optimization" (2015), Algorithm 1, with the bias corrections applied to the moments.

Pins (tests): central finite differences of `loss` against `loss_grad`; the all-active case,
where the network is one affine map; the all-inactive case; Adam's first step, which moves every
parameter by lr * sign(g) up to eps.
"""
import numpy as np

IN, HID = 3, 64


def n_params(n_out, n_in=IN, n_hid=HID):
    return n_hid * n_in + n_hid + n_hid * n_hid + n_hid + n_out * n_hid + n_out


def unpack(theta, n_out, n_in=IN, n_hid=HID):
    """The flat parameter vector as (W1, b1, W2, b2, W3, b3) float64 views."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == n_params(n_out, n_in, n_hid)
    shapes = [(n_hid, n_in), (n_hid,), (n_hid, n_hid), (n_hid,), (n_out, n_hid), (n_out,)]
    out, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(theta[o:o + k].reshape(sh))
        o += k
    return out


def forward(theta, X, n_out, n_in=IN, n_hid=HID):
    """Outputs y[n][n_out] and the activations (z1, h1, z2, h2) for inputs X[n][n_in]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_out, n_in, n_hid)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (z1, h1, z2, h2)


def loss(theta, X, T, mask, mask_sum, n_out, n_in=IN, n_hid=HID):
    y, _ = forward(theta, X, n_out, n_in, n_hid)
    return float(np.sum(np.asarray(mask, np.float64) * (y - T) ** 2) / mask_sum)


def loss_grad(theta, X, T, mask, mask_sum, n_out, n_in=IN, n_hid=HID):
    """(loss, gradient as a flat vector in the parameter order) by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_out, n_in, n_hid)
    X = np.asarray(X, dtype=np.float64)
    mask = np.asarray(mask, dtype=np.float64)
    y, (z1, h1, z2, h2) = forward(theta, X, n_out, n_in, n_hid)
    L = float(np.sum(mask * (y - T) ** 2) / mask_sum)
    dy = 2.0 * mask * (y - T) / mask_sum              # dL/dy
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return L, g


def adam_step(theta, g, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns new (theta, m1, m2).  step counts from 1."""
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    mhat = m1 / (1 - beta1 ** step)
    vhat = m2 / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def features(a_bits, b_bits, batch):
    """Selector inputs: (log2(longer) - 21)/9, (log2(shorter) - 21)/9, log2(batch)/12, with bit
    counts rounded up to whole 32-bit limbs (at least one)."""
    la = 32.0 * max(1, -(-int(a_bits) // 32))
    lb = 32.0 * max(1, -(-int(b_bits) // 32))
    return np.array([(np.log2(max(la, lb)) - 21.0) / 9.0, (np.log2(min(la, lb)) - 21.0) / 9.0,
                     np.log2(float(batch)) / 12.0])
