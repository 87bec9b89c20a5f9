"""Reference of the null-vector proposal network (oracle; test infrastructure only).

Plain FP64 NumPy forward and backward of the small local CNN that proposes
initial near-null vectors for the adaptive setup, the block-local gauge fixing
it works in, and the projection loss it is trained with.  The adaptive
procedure of the paper defines what the network imitates (its targets are the
vectors that the adaptive setup produces); the network itself is not part of
the paper.

Architecture: four 3x3 convolutions with periodic (circular) padding,
channels 4 -> 64 -> 64 -> 64 -> 32, tanh between layers, none after the last.
Input channels per site: cos/sin of the two link angles (theta_1, theta_2)
after block-local tree gauge fixing.  Output channels per site: 8 complex
vectors x 2 spin components x (re, im), channel index 4k + 2s + c.

Arrays are NCHW with H = x_2 (rows) and W = x_1 (columns).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (4, 64, 64, 64, 32)


def init_params(rng: np.random.Generator, channels=CHANNELS):
    """He-style initialisation; weights W[l] of shape (C_out, C_in, 3, 3), biases (C_out,)."""
    params = []
    for ci, co in zip(channels[:-1], channels[1:]):
        W = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(1.0 / (9 * ci))
        b = np.zeros(co)
        params.append((W, b))
    return params


def n_params(params) -> int:
    return int(sum(W.size + b.size for W, b in params))


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n, o, i, j] = b[o] + sum_{c, di, dj} W[o, c, di, dj] x[n, c, i + di - 1, j + dj - 1] (periodic)."""
    y = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for di in range(3):
        for dj in range(3):
            xs = np.roll(x, shift=(1 - di, 1 - dj), axis=(2, 3))     # xs[i, j] = x[i + di - 1, j + dj - 1]
            y += np.einsum("oc,ncij->noij", W[:, :, di, dj], xs)
    return y + b[None, :, None, None]


def conv3x3_backward(x: np.ndarray, W: np.ndarray, dy: np.ndarray):
    """Gradients (dx, dW, db) of conv3x3 for upstream gradient dy."""
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    for di in range(3):
        for dj in range(3):
            xs = np.roll(x, shift=(1 - di, 1 - dj), axis=(2, 3))
            dW[:, :, di, dj] = np.einsum("noij,ncij->oc", dy, xs)
            dxs = np.einsum("oc,noij->ncij", W[:, :, di, dj], dy)
            dx += np.roll(dxs, shift=(di - 1, dj - 1), axis=(2, 3))
    db = dy.sum(axis=(0, 2, 3))
    return dx, dW, db


def forward(params, x: np.ndarray):
    """Network output and the activations needed by backward."""
    acts = [x]
    h = x
    for l, (W, b) in enumerate(params):
        z = conv3x3(h, W, b)
        h = np.tanh(z) if l < len(params) - 1 else z
        acts.append(h)
    return h, acts


def backward(params, acts, dout: np.ndarray):
    """Gradients [(dW, db), ...] for d(loss)/d(output) = dout."""
    grads = [None] * len(params)
    g = dout
    for l in reversed(range(len(params))):
        W, _ = params[l]
        if l < len(params) - 1:
            g = g * (1.0 - acts[l + 1] ** 2)            # tanh'
        dx, dW, db = conv3x3_backward(acts[l], W, g)
        grads[l] = (dW, db)
        g = dx
    return grads


# ----------------------------------------------------------------------------
# block-local tree gauge
# ----------------------------------------------------------------------------

def tree_gauge_phase(theta: np.ndarray, block=(4, 4)) -> np.ndarray:
    """Phase phi(x) of the gauge transformation g = exp(i phi) that sets to 1 a
    maximal tree of links inside every block: the x_1-links along each row of
    the block and the x_2-links along the block's first column.  phi = 0 at
    the block origin.  theta: (2, L2, L1); returns (L2, L1)."""
    L2, L1 = theta.shape[1:]
    b1, b2 = block
    phi = np.zeros((L2, L1))
    for y in range(L2):
        yb = y % b2
        for x in range(L1):
            xb = x % b1
            if xb == 0:
                phi[y, x] = 0.0 if yb == 0 else phi[y - 1, x] + theta[1, y - 1, x]
            else:
                phi[y, x] = phi[y, x - 1] + theta[0, y, x - 1]
    return phi


def gauge_transform_u1(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """theta'_mu(x) = phi(x) + theta_mu(x) - phi(x + mu), wrapped to (-pi, pi]."""
    t = np.empty_like(theta)
    t[0] = phi + theta[0] - np.roll(phi, -1, axis=1)
    t[1] = phi + theta[1] - np.roll(phi, -1, axis=0)
    return np.angle(np.exp(1j * t))


def network_input(theta: np.ndarray) -> np.ndarray:
    """(4, L2, L1): cos theta_1, sin theta_1, cos theta_2, sin theta_2."""
    return np.stack([np.cos(theta[0]), np.sin(theta[0]), np.cos(theta[1]), np.sin(theta[1])])


def output_to_vectors(out: np.ndarray, nvec: int = 8) -> np.ndarray:
    """(32, L2, L1) network output -> (nvec, L2*L1, 2) complex vectors."""
    C, L2, L1 = out.shape
    o = out.reshape(nvec, 2, 2, L2 * L1)
    return np.transpose(o[:, :, 0] + 1j * o[:, :, 1], (0, 2, 1))


def vectors_to_output(v: np.ndarray) -> np.ndarray:
    """Inverse of output_to_vectors for gradients: complex (nvec, V, 2) -> real (4 nvec, V)."""
    nvec, V, _ = v.shape
    o = np.zeros((nvec, 2, 2, V))
    o[:, :, 0] = np.transpose(v.real, (0, 2, 1))
    o[:, :, 1] = np.transpose(v.imag, (0, 2, 1))
    return o.reshape(4 * nvec, V)


# ----------------------------------------------------------------------------
# projection loss on the chirally split block spans
# ----------------------------------------------------------------------------

def projection_loss(pred: np.ndarray, target: np.ndarray, dims, block=(4, 4), eps: float = 1e-3):
    """Loss and d(loss)/d(conj pred) for complex vectors (nvec, V, 2).

    For every block S_j and chirality s (spin component s in two dimensions),
    with V_p the block-restricted predicted vectors (columns) and t_k the
    target ones: L_js = sum_k (1 - t_k^dag Pi t_k / ||t_k||^2) with
    Pi = V_p (V_p^dag V_p + eps 1)^-1 V_p^dag, which at eps = 0 is the
    squared relative distance ||(1 - Pi) t_k||^2 / ||t_k||^2 of t_k from the
    predicted span.  The loss is the mean over (blocks, chiralities, target
    vectors).  The span, not the basis, is what
    the prolongator uses, so the loss is invariant under any invertible mixing
    of the predicted vectors within a block (up to eps).

    With S = sum_k t_k t_k^dag/||t_k||^2, G = V^dag V + eps and
    A = G^-1 V^dag S V G^-1:  dL/d(conj V) = -S V G^-1 + V A (per block).
    """
    L1, L2 = dims
    b1, b2 = block
    nvec = pred.shape[0]
    x2, x1 = np.meshgrid(np.arange(L2), np.arange(L1), indexing="ij")
    blk = ((x2 // b2) * (L1 // b1) + x1 // b1).ravel()
    nb = blk.max() + 1
    loss = 0.0
    grad = np.zeros_like(pred)
    count = 0
    for j in range(nb):
        sites = np.nonzero(blk == j)[0]
        for s in range(2):
            Vp = pred[:, sites, s].T                     # (bs, nvec)
            T = target[:, sites, s].T
            tn = T / np.linalg.norm(T, axis=0, keepdims=True)
            S = tn @ tn.conj().T
            G = Vp.conj().T @ Vp + eps * np.eye(nvec)
            Gi = np.linalg.inv(G)
            Pi = Vp @ Gi @ Vp.conj().T
            loss += float(np.real(np.trace(S) - np.trace(Pi @ S)))
            A = Gi @ Vp.conj().T @ S @ Vp @ Gi
            g = -S @ Vp @ Gi + Vp @ A
            grad[:, sites, s] = g.T
            count += T.shape[1]
    return loss / count, grad / count


def loss_and_param_grads(params, theta_fixed: np.ndarray, target_fixed: np.ndarray, block=(4, 4), eps=1e-3):
    """Full pipeline for one configuration (in the tree gauge): loss and parameter gradients.

    Real gradients follow from the Wirtinger derivative: dL/dRe = 2 Re g, dL/dIm = 2 Im g.
    """
    L2, L1 = theta_fixed.shape[1:]
    x = network_input(theta_fixed)[None]
    out, acts = forward(params, x)
    pred = output_to_vectors(out[0])
    loss, g = projection_loss(pred, target_fixed, (L1, L2), block, eps)
    dout = vectors_to_output(2.0 * g).reshape(out.shape)
    return loss, backward(params, acts, dout)
