"""Oracle: the schedule selector's multilayer perceptron in float64.  TEST INFRASTRUCTURE ONLY.

The paper observes that the minimal number of passes is not always the fastest plan and
proposes minimising a model of the true cost instead (Sec. 5; Sec. 4.2 on the effect of
large extents).  The selector realises that model as a small fully connected
network 40 -> 64 -> 64 -> 6 with ReLU after the two hidden layers, predicting the base-2
logarithm of the run time (ms) of each of six candidate schedules; it is trained by
minimising the mean squared error (a target that is not a number -- a candidate that does not
exist for that request -- contributes zero) with Adam (Kingma and Ba, "Adam: A Method for
Stochastic Optimization", ICLR 2015, Algorithm 1).

Parameter vector layout (float, 7174 entries): W1 (64 x 40, row-major: W1[o, i]), b1 (64),
W2 (64 x 64), b2 (64), W3 (6 x 64), b3 (6).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the 64-bit variant published by Vigna), so that the
initial weights and the minibatch order can be reproduced exactly from a seed.
Parity: pinned by central finite differences of the loss, closed forms (zero weights give
the last bias; a zero-loss dataset leaves Adam still), Adam's first-step property
(|step| = learning rate) and the published SplitMix64 outputs.
"""
import numpy as np

SIZES = (40, 64, 64, 6)
MASK64 = (1 << 64) - 1


def layout():
    """[(name, shape, offset)] of the flat parameter vector."""
    out, off = [], 0
    for li in range(3):
        fan_in, fan_out = SIZES[li], SIZES[li + 1]
        out.append((f"W{li + 1}", (fan_out, fan_in), off))
        off += fan_in * fan_out
        out.append((f"b{li + 1}", (fan_out,), off))
        off += fan_out
    return out, off


LAYOUT, NPARAM = layout()


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return {name: theta[off:off + int(np.prod(shape))].reshape(shape) for name, shape, off in LAYOUT}


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _, _ in LAYOUT])


class SplitMix64:
    """SplitMix64: state += 0x9E3779B97F4A7C15, then the two xor-shift-multiply rounds."""

    def __init__(self, seed):
        self.state = int(seed) & MASK64

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        """Double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def init_params(seed):
    """Weights uniform in [-a, a] with a = sqrt(6 / fan_in) (He et al. 2015, uniform form),
    biases zero; drawn in layout order, row-major.  Rounded to float32 like the device copy."""
    rng = SplitMix64(seed)
    theta = np.zeros(NPARAM)
    for name, shape, off in LAYOUT:
        if name.startswith("W"):
            a = np.sqrt(6.0 / shape[1])
            for k in range(shape[0] * shape[1]):
                theta[off + k] = (2.0 * rng.uniform() - 1.0) * a
    return theta.astype(np.float32).astype(np.float64)


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, X):
    """Hidden activations and outputs: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
    y = W3 h2 + b3, for every row x of X."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = relu(X @ p["W1"].T + p["b1"])
    h2 = relu(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return h1, h2, y


def _errors(y, T):
    """y - T where the target is a number, 0 where it is not."""
    T = np.asarray(T, dtype=np.float64)
    return np.where(np.isnan(T), 0.0, y - np.where(np.isnan(T), 0.0, T))


def loss(theta, X, T):
    """Mean over rows and outputs of the squared error (NaN targets contribute zero)."""
    _, _, y = forward(theta, X)
    return float(np.mean(_errors(y, T) ** 2))


def backward(theta, X, T):
    """(loss, gradient of the loss with respect to theta), by the chain rule layer by layer."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1, h2, y = forward(theta, X)
    n = X.shape[0]
    e = _errors(y, T)
    d3 = 2.0 * e / (n * SIZES[3])                # dL/dy
    g = {"W3": d3.T @ h2, "b3": d3.sum(axis=0)}
    d2 = (d3 @ p["W3"]) * (h2 > 0)               # dL/d(pre-activation of layer 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (h1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    return float(np.mean(e ** 2)), pack(g)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def epoch_order(rng, n):
    """A uniformly random permutation of 0..n-1 (Fisher-Yates, j = next() mod (i + 1))."""
    idx = list(range(n))
    for i in range(n - 1, 0, -1):
        j = rng.next() % (i + 1)
        idx[i], idx[j] = idx[j], idx[i]
    return idx


def train(theta, X, T, epochs, batch, lr, seed, beta1=0.9, beta2=0.999, eps=1e-8):
    """Minibatch Adam: every epoch visits the rows in a fresh random order, in batches of
    `batch` rows (the last one may be shorter).  Returns (theta, loss of the last batch)."""
    theta = np.array(theta, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)  # NaN entries: no target
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    rng = SplitMix64(seed)
    step, last = 0, None
    for _ in range(epochs):
        order = epoch_order(rng, X.shape[0])
        for s in range(0, len(order), batch):
            rows = order[s:s + batch]
            last, g = backward(theta, X[rows], T[rows])
            step += 1
            theta, m, v = adam_step(theta, g, m, v, step, lr, beta1, beta2, eps)
    return theta, last
