"""Reference of the learned per-block codec selector's network, in float64
numpy (test infrastructure: only tests, the smoke check and the CPU baseline
use it; the product path never does).

Network: 40 features -> 64 -> 64 -> 16 class logits, ReLU between layers,
softmax.  The selector is not part of the paper; its classes are the
per-block codec classes of the oracle's block container.

The device computes with bf16 matrix operands and fp32 accumulation; with
``bf=True`` this reference rounds to bf16 (round to nearest even, 8
significant bits) at exactly the points where the device does, and computes
everything else in float64:

  forward   A0 = bf(X); Z1 = A0 bf(W1) + b1; A1 = bf(relu(Z1));
            Z2 = A1 bf(W2) + b2;  A2 = bf(relu(Z2)); Z3 = A2 bf(W3) + b3;
            P = softmax(Z3)
  loss      mean over rows of  -log P[y]  +  lam * sum_k P_k c_k
            (c_k >= 0: the relative size excess of class k over the block's
            least size, so the second term is the expected excess)
  backward  G3 = (P - onehot(y) + lam P (c - <P, c>)) / B
            dW3 = A2^T bf(G3);  db3 = sum G3;  dA2 = bf(G3) bf(W3)^T
            dZ2 = dA2 [A2 > 0]; dW2 = A1^T bf(dZ2); db2 = sum dZ2
            dA1 = bf(dZ2) bf(W2)^T
            dZ1 = dA1 [A1 > 0]; dW1 = A0^T bf(dZ1); db1 = sum dZ1

With ``bf=False`` nothing is rounded and the gradient is the exact gradient
of the loss (pinned by central finite differences).  Adam is the textbook
update with bias correction."""
import numpy as np

NF, NH, NC = 40, 64, 16
SHAPES = [("W1", (NF, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NC)), ("b3", (NC,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x):
    """Round to the nearest bfloat16 (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


def unflatten(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == NPARAM
    out, o = {}, 0
    for name, s in SHAPES:
        k = int(np.prod(s))
        out[name] = theta[o:o + k].reshape(s)
        o += k
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed):
    """He-normal weights, zero biases, as float32 values."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, s in SHAPES:
        if name[0] == "W":
            p[name] = rng.normal(0.0, np.sqrt(2.0 / s[0]), s)
        else:
            p[name] = np.zeros(s)
    return flatten(p).astype(np.float32)


def forward(theta, X, bf=True):
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    p = unflatten(theta)
    f = {}
    f["A0"] = r(X)
    f["Z1"] = f["A0"] @ r(p["W1"]) + p["b1"]
    f["A1"] = r(np.maximum(f["Z1"], 0.0))
    f["Z2"] = f["A1"] @ r(p["W2"]) + p["b2"]
    f["A2"] = r(np.maximum(f["Z2"], 0.0))
    f["Z3"] = f["A2"] @ r(p["W3"]) + p["b3"]
    z = f["Z3"] - f["Z3"].max(axis=1, keepdims=True)
    e = np.exp(z)
    f["P"] = e / e.sum(axis=1, keepdims=True)
    f["logZ"] = np.log(e.sum(axis=1)) + f["Z3"].max(axis=1)
    return f


def loss(theta, X, y, c=None, lam=0.0, bf=True):
    f = forward(theta, X, bf)
    B = X.shape[0]
    ce = f["logZ"] - f["Z3"][np.arange(B), y]
    tot = ce.sum()
    if lam:
        tot += lam * (f["P"] * c).sum()
    return tot / B


def grad(theta, X, y, c=None, lam=0.0, bf=True):
    """(mean loss, flat gradient) of the batch."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    p = unflatten(theta)
    f = forward(theta, X, bf)
    B = X.shape[0]
    P = f["P"]
    onehot = np.zeros_like(P)
    onehot[np.arange(B), y] = 1.0
    G3 = P - onehot
    L = (f["logZ"] - f["Z3"][np.arange(B), y]).sum()
    if lam:
        c = np.asarray(c, dtype=np.float64)
        ec = (P * c).sum(axis=1, keepdims=True)
        G3 = G3 + lam * P * (c - ec)
        L += lam * ec.sum()
    G3 = G3 / B
    g = {}
    g["W3"] = f["A2"].T @ r(G3)
    g["b3"] = G3.sum(axis=0)
    dA2 = r(G3) @ r(p["W3"]).T
    dZ2 = dA2 * (f["A2"] > 0)
    g["W2"] = f["A1"].T @ r(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dA1 = r(dZ2) @ r(p["W2"]).T
    dZ1 = dA1 * (f["A1"] > 0)
    g["W1"] = f["A0"].T @ r(dZ1)
    g["b1"] = dZ1.sum(axis=0)
    return L / B, flatten(g)


def predict(theta, X, bf=True):
    """Class of every row: the first index of the largest logit."""
    return np.argmax(forward(theta, X, bf)["Z3"], axis=1)


class Adam:
    """Adam with bias correction over a flat parameter vector."""

    def __init__(self, theta, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.theta = np.asarray(theta, dtype=np.float64).copy()
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        self.theta = self.theta - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.theta
