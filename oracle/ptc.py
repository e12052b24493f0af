"""FP64 oracle of the parallel-transport convolution (PTC) preconditioner -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU leg import this module.

A PTC layer maps C_in spinor fields to C_out spinor fields:

    out[a](x) = sum_b sum_p  W_p^{ab} (T_p in[b])(x)

with nine paths p: the identity (p = 0) and the eight one-hop parallel
transports (p = 1 + 2 mu for +mu, p = 2 + 2 mu for -mu):

    (T_{+mu} psi)(x) = U_mu(x)           psi(x + mu)
    (T_{-mu} psi)(x) = U_mu(x - mu)^+    psi(x - mu)

the transports carrying the same boundary phases as the Wilson operator (z_mu
on a wrapped forward hop, conj(z_mu) on a wrapped backward hop).  Each W_p^{ab}
is a complex 4x4 matrix acting on spin; the transports act on colour and site,
so the two commute.  The network is two such layers (1 -> C hidden channels ->
1), linear, without bias: the target D^-1 is linear and a bias would break gauge
covariance.  With W_{+mu} = 1 - gamma_mu, W_{-mu} = 1 + gamma_mu, W_0 = 0 one
layer is exactly the hopping term H of Eq. (1).

Weights are arrays of shape (9, C_out, C_in, 4, 4) complex128; fields are
canonical (Lt, Lz, Ly, Lx, 4, 3) complex128, a list per channel.

Gradients follow the Wirtinger convention for a real loss L: for a linear map
out = A(in), g_out = dL/d conj(out) gives dL/d conj(in) = A^+(g_out) and
dL/d conj(W_p^{ab}) = sum_x,colour g_out[a](x) (T_p in[b])(x)^+.
"""

from __future__ import annotations

import numpy as np

NPATH = 9
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # direction mu -> array axis of (t, z, y, x, ...)


def path_of(p: int):
    """p -> (mu, sign) for p >= 1; (None, 0) for the identity."""
    if p == 0:
        return None, 0
    mu = (p - 1) // 2
    return mu, (+1 if (p - 1) % 2 == 0 else -1)


def reverse_path(p: int) -> int:
    if p == 0:
        return 0
    return p + 1 if (p - 1) % 2 == 0 else p - 1


def _edge(field, axis, index):
    sl = [slice(None)] * field.ndim
    sl[axis] = index
    return tuple(sl)


def transport(psi, gauge, phases, p):
    """(T_p psi)(x) for one spinor field."""
    mu, sgn = path_of(p)
    if mu is None:
        return psi.copy()
    ax = _AXIS[mu]
    z = complex(np.asarray(phases, dtype=np.complex128).reshape(4)[mu])
    u = gauge[..., mu, :, :]
    if sgn > 0:
        nb = np.roll(psi, -1, axis=ax)                      # psi(x + mu)
        nb[_edge(nb, ax, psi.shape[ax] - 1)] *= z           # wrapped forward hop
        return np.einsum("...ij,...sj->...si", u, nb)
    nb = np.roll(psi, 1, axis=ax)                           # psi(x - mu)
    nb[_edge(nb, ax, 0)] *= np.conj(z)                      # wrapped backward hop
    ub = np.roll(u, 1, axis=ax)                             # U_mu(x - mu)
    return np.einsum("...ji,...sj->...si", np.conj(ub), nb)


def layer(inputs, weights, gauge, phases):
    """out[a] = sum_b sum_p W_p^{ab} T_p in[b]."""
    npath, cout, cin = weights.shape[:3]
    assert npath == NPATH and len(inputs) == cin
    out = [np.zeros_like(inputs[0]) for _ in range(cout)]
    for p in range(NPATH):
        for b in range(cin):
            t = transport(inputs[b], gauge, phases, p)
            for a in range(cout):
                out[a] += np.einsum("st,...tc->...sc", weights[p, a, b], t)
    return out


def layer_adjoint(grads, weights, gauge, phases):
    """Adjoint of `layer` (as a linear map of its inputs): g_in[b] = sum_a sum_p T_p^+ W_p^{ab +} g_out[a].

    T_{+mu}^+ = T_{-mu}: the adjoint of a transport is the reverse transport.
    """
    npath, cout, cin = weights.shape[:3]
    assert len(grads) == cout
    out = [np.zeros_like(grads[0]) for _ in range(cin)]
    for p in range(NPATH):
        for a in range(cout):
            for b in range(cin):
                mixed = np.einsum("ts,...tc->...sc", np.conj(weights[p, a, b]), grads[a])
                out[b] += transport(mixed, gauge, phases, reverse_path(p))
    return out


def weight_grad(grads, inputs, gauge, phases):
    """dL/d conj(W_p^{ab}) = sum_x sum_colour g_out[a](x) (T_p in[b])(x)^+, shape (9, C_out, C_in, 4, 4)."""
    cout, cin = len(grads), len(inputs)
    g = np.zeros((NPATH, cout, cin, 4, 4), dtype=np.complex128)
    for p in range(NPATH):
        for b in range(cin):
            t = transport(inputs[b], gauge, phases, p)
            for a in range(cout):
                g[p, a, b] = np.einsum("nsc,ntc->st", grads[a].reshape(-1, 4, 3), np.conj(t).reshape(-1, 4, 3))
    return g


def net_apply(r, w1, w2, gauge, phases):
    """Two-layer network M(r) (1 -> C -> 1 channels). Returns (output field, hidden fields)."""
    hidden = layer([r], w1, gauge, phases)
    return layer(hidden, w2, gauge, phases)[0], hidden


def net_backward(g_out, r, hidden, w2, gauge, phases):
    """Weight gradients of the two-layer network from g_out = dL/d conj(M(r)): (dL/dW1*, dL/dW2*)."""
    g2 = weight_grad([g_out], hidden, gauge, phases)
    g_hidden = layer_adjoint([g_out], w2, gauge, phases)
    g1 = weight_grad(g_hidden, [r], gauge, phases)
    return g1, g2


def loss_and_grads(pairs, w1, w2, gauge, phases):
    """L = (1/N) sum_i ||M(r_i) - e_i||^2 / ||e_i||^2 and its Wirtinger gradients (dL/dW1*, dL/dW2*).

    pairs: list of (r_i, e_i) on this gauge field."""
    n = len(pairs)
    loss = 0.0
    g1 = np.zeros_like(w1)
    g2 = np.zeros_like(w2)
    for r, e in pairs:
        out, hidden = net_apply(r, w1, w2, gauge, phases)
        en = float(np.sum(np.abs(e) ** 2))
        d = out - e
        loss += float(np.sum(np.abs(d) ** 2)) / en / n
        a, b = net_backward(d / (en * n), r, hidden, w2, gauge, phases)
        g1 += a
        g2 += b
    return loss, g1, g2


def loss_and_grads_residual(residuals, w1, w2, gauge, phases, kappa):
    """Residual-norm loss L = (1/N) sum_i ||D M(r_i) - r_i||^2 / ||r_i||^2 and its gradients.

    For a training pair (r, e) with r = D e this is ||D (M(r) - e)||^2 / ||D e||^2:
    the error of M(r) as an estimate of e, measured by the residual it leaves,
    which is what one step x += M(r) of a right-preconditioned Krylov method
    reduces.  With y = D M(r) - r, dL/d conj(M(r)) = D^+ y / (N ||r||^2)."""
    from . import oracle as orc

    n = len(residuals)
    loss = 0.0
    g1 = np.zeros_like(w1)
    g2 = np.zeros_like(w2)
    for r in residuals:
        out, hidden = net_apply(r, w1, w2, gauge, phases)
        rn = float(np.sum(np.abs(r) ** 2))
        y = orc.dirac(out, gauge, kappa, phases) - r
        loss += float(np.sum(np.abs(y) ** 2)) / rn / n
        g_out = orc.dirac(y, gauge, kappa, phases, dagger=True) / (rn * n)
        a, b = net_backward(g_out, r, hidden, w2, gauge, phases)
        g1 += a
        g2 += b
    return loss, g1, g2


def adam_step(w, g_conj, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on complex weights viewed as (Re, Im) real parameters.

    The gradient of L w.r.t. (Re W, Im W) is (2 Re G, 2 Im G) with G = dL/dW*.
    m, v: real arrays of shape w.shape + (2,). Returns the updated (w, m, v)."""
    grad = np.stack([2 * g_conj.real, 2 * g_conj.imag], axis=-1)
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    step = lr * mh / (np.sqrt(vh) + eps)
    w = w - (step[..., 0] + 1j * step[..., 1])
    return w, m, v
