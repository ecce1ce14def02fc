"""Float64 reference of the precision-proposal network (TEST INFRASTRUCTURE).

The network maps a feature vector (N, beta, ln N), scaled by the caller, to
two outputs (scaled required precision in bits, scaled ln lambda_1):

    h1 = relu(W1 x + b1)      64 units
    h2 = relu(W2 h1 + b2)     64 units
    h3 = relu(W3 h2 + b3)     64 units
    y  = W4 h3 + b4           2 outputs

trained by mean squared error with Adam (Kingma & Ba, "Adam: a method for
stochastic optimization", 2015, Algorithm 1: bias-corrected first and second
moment estimates).  Parameters are one packed vector in the order
[W1 (64x3), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (2x64), b4], each matrix
row-major with shape (outputs, inputs).

Pins (tests/test_oracle_mlp.py): the backward pass against central finite
differences of the loss in float64; a network whose pre-activations are all
positive equals the product of its affine maps; the first Adam step moves
every parameter with a nonzero gradient by exactly lr * sign(g) (up to eps);
the MSE gradient against its finite difference.
"""
import numpy as np

NI, NH, NO = 3, 64, 2
SHAPES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NO, NH)), ("b4", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Views of the packed parameter vector, by name."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


def init(seed):
    """He-uniform initial weights, zero biases (float64; cast by the caller)."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            parts[name] = rng.uniform(-lim, lim, size=shp)
        else:
            parts[name] = np.zeros(shp)
    return pack(parts)


def forward(theta, X):
    """Outputs (batch x 2) and the activations the backward pass needs."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    h3 = np.maximum(h2 @ p["W3"].T + p["b3"], 0.0)
    Y = h3 @ p["W4"].T + p["b4"]
    return Y, (X, h1, h2, h3)


def mse(Y, T):
    """Mean of the squared errors over all batch x 2 outputs, and dL/dY."""
    D = np.asarray(Y, dtype=np.float64) - np.asarray(T, dtype=np.float64)
    return float(np.mean(D * D)), 2.0 * D / D.size


def backward(theta, acts, dY):
    """Gradient of sum(dY * Y) with respect to the packed parameters (chain
    rule through the affine maps; the ReLU passes where its output is > 0)."""
    p = unpack(theta)
    X, h1, h2, h3 = acts
    dY = np.asarray(dY, dtype=np.float64)
    g = {"W4": dY.T @ h3, "b4": dY.sum(0)}
    d3 = (dY @ p["W4"]) * (h3 > 0)
    g["W3"], g["b3"] = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ p["W3"]) * (h2 > 0)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (h1 > 0)
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return pack(g)


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, T, steps, lr, batch=None, seed=0):
    """Full-batch (or seeded mini-batch) Adam on the MSE; returns theta and
    the loss history."""
    rng = np.random.default_rng(seed)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, steps + 1):
        idx = slice(None) if batch is None else rng.choice(len(X), batch, replace=False)
        Y, acts = forward(theta, X[idx])
        loss, dY = mse(Y, T[idx])
        hist.append(loss)
        theta, m, v = adam_step(theta, m, v, backward(theta, acts, dY), t, lr)
    return theta, hist
