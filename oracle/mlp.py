"""FP64 reference of the cost model's network: a ReLU MLP, its MSE loss, the
gradients by the chain rule, and one Adam step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network (a project addition; the Tiramisu paper only motivates a precise
cost model, Sections I and II):
  dims = [F, H1, ..., 1]; layer l maps A_{l-1} (rows x dims[l]) to
  Z_l = A_{l-1} W_l + b_l with W_l of shape dims[l] x dims[l+1];
  A_l = relu(Z_l) for every layer but the last, whose Z is the output.
Parameters are stored as one flat vector, layer by layer: W_l row-major,
then b_l.
Loss: mean squared error L = (1/n) sum_i (out_i - y_i)^2.
Gradients: dOut = 2 (out - y) / n; for each layer from the last,
  dZ_l = dA_l * [Z_l > 0] (hidden layers; the derivative of relu at 0 is
  taken as 0), dW_l = A_{l-1}^T dZ_l, db_l = column sums of dZ_l,
  dA_{l-1} = dZ_l W_l^T.
Adam (Kingma and Ba, 2015): with step t >= 1,
  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
  p = p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def param_count(dims):
    return sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(len(dims) - 1))


def unpack(params, dims):
    """[(W_l, b_l)] views into the flat parameter vector."""
    out, off = [], 0
    for l in range(len(dims) - 1):
        w = params[off:off + dims[l] * dims[l + 1]].reshape(dims[l], dims[l + 1])
        off += dims[l] * dims[l + 1]
        b = params[off:off + dims[l + 1]]
        off += dims[l + 1]
        out.append((w, b))
    return out


def forward(params, dims, X):
    """(output vector, list of activations A_{-1}=X, A_0, ..., Z_last)."""
    params = np.asarray(params, dtype=np.float64)
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(params, dims)
    for l, (w, b) in enumerate(layers):
        z = acts[-1] @ w + b
        if l < len(layers) - 1:
            z = np.maximum(z, 0.0)
        acts.append(z)
    return acts[-1][:, 0], acts


def loss(params, dims, X, y):
    out, _ = forward(params, dims, X)
    d = out - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def gradients(params, dims, X, y):
    """(loss, flat gradient vector) in FP64."""
    params = np.asarray(params, dtype=np.float64)
    out, acts = forward(params, dims, X)
    n = len(out)
    y = np.asarray(y, dtype=np.float64)
    L = float(np.mean((out - y) ** 2))
    layers = unpack(params, dims)
    grads = [None] * len(layers)
    dA = (2.0 * (out - y) / n)[:, None]
    for l in range(len(layers) - 1, -1, -1):
        w, _ = layers[l]
        if l < len(layers) - 1:
            dZ = dA * (acts[l + 1] > 0.0)
        else:
            dZ = dA
        gW = acts[l].T @ dZ
        gb = dZ.sum(axis=0)
        grads[l] = (gW, gb)
        dA = dZ @ w.T
    flat = np.concatenate([np.concatenate([g.ravel(), b]) for g, b in grads])
    return L, flat


def adam_step(params, grads, m, v, step, lr):
    """One Adam update; returns (params, m, v) as new FP64 arrays."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grads, dtype=np.float64)
    m = BETA1 * np.asarray(m, dtype=np.float64) + (1.0 - BETA1) * g
    v = BETA2 * np.asarray(v, dtype=np.float64) + (1.0 - BETA2) * g * g
    mhat = m / (1.0 - BETA1 ** step)
    vhat = v / (1.0 - BETA2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + EPS), m, v
