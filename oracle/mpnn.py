"""Float64 reference of the learned diagonal preconditioner's network (TEST INFRASTRUCTURE).

The paper uses the Jacobi preconditioner M = diag(K) for K = P̄ + σI + ρ̄ĀᵀĀ (Section 6.3.1).
The learned variant keeps M diagonal and strictly positive, so PCG stays a valid Algorithm 3:

    M⁻¹_ii = softplus(g_i) / K_ii,

where g is produced by a message-passing network over the bipartite variable/constraint graph
of Ā. softplus(g) = 1 reproduces Jacobi exactly. The output layer is initialised there.

Architecture (hidden width 32, L rounds):
  inputs   f_v ∈ ℝ^{n×32}, f_c ∈ ℝ^{m×32}   (4 features each, zero-padded to 32)
  h_v⁰ = relu(f_v W_v0 + b_v0),  h_c⁰ = relu(f_c W_c0 + b_c0)
  round ℓ: a_c = Â h_v^{ℓ−1};  h_c^ℓ = relu([h_c^{ℓ−1}, a_c] W_cℓ + b_cℓ)
           a_v = Ǎ h_c^ℓ;      h_v^ℓ = relu([h_v^{ℓ−1}, a_v] W_vℓ + b_vℓ)
  head:    u = relu([h_v^L, φ] W_h1 + b_h1);  g = u w_h2 + b_h2
with Â_ji = |Ā_ji| / Σ_i |Ā_ji| (rows of Ā normalised), Ǎ_ij = |Ā_ji| / Σ_j |Ā_ji| (columns).

Node features (on the Ruiz-scaled data):
  variable i:   log(P̄_ii + σ), log(‖Ā_i‖² + 1e-12), log(1 + deg_i), log(max_j |Ā_ji| + 1e-12)
  constraint j: log(‖Ā_j‖² + 1e-12), log(1 + deg_j), [l_j = u_j], log(max_i |Ā_ji| + 1e-12)
  head, depends on ρ̄: φ = (log(ρ̄‖Ā_i‖² + 1e-12) − log K_ii, log(P̄_ii + σ) − log K_ii).
Only the head sees ρ̄, so a ρ̄ change re-evaluates just the head.

Loss against Hutchinson estimates ĥ of diag(K⁻¹) (clamped at 1/K_ii, since (K⁻¹)_ii ≥ 1/K_ii
for SPD K): the mean-removed squared error of log M⁻¹_ii − log ĥ_i, i.e. with
e_i = log softplus(g_i) − log(ĥ_i K_ii):  L = mean_i (e_i − ē)².
PCG is invariant to scaling M, hence the mean removal.

Flat parameter layout (float32, row-major; this layout is the interface the device code also
reads): W_v0[32×32], b_v0[32], W_c0[32×32], b_c0[32], then for ℓ = 1..L: W_cℓ[64×32], b_cℓ[32],
W_vℓ[64×32], b_vℓ[32]; then W_h1[64×32], b_h1[32], w_h2[32], b_h2[1].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

H = 32
ROUNDS = 3
INIT_BIAS = float(np.log(np.e - 1.0))  # softplus(INIT_BIAS) = 1


def layout(rounds=ROUNDS):
    """List of (name, shape) in flat order."""
    out = [("W_v0", (32, H)), ("b_v0", (H,)), ("W_c0", (32, H)), ("b_c0", (H,))]
    for l in range(1, rounds + 1):
        out += [(f"W_c{l}", (2 * H, H)), (f"b_c{l}", (H,)), (f"W_v{l}", (2 * H, H)), (f"b_v{l}", (H,))]
    out += [("W_h1", (2 * H, H)), ("b_h1", (H,)), ("w_h2", (H,)), ("b_h2", (1,))]
    return out


def nparams(rounds=ROUNDS):
    return int(sum(np.prod(s) for _, s in layout(rounds)))


def unpack(theta, rounds=ROUNDS):
    theta = np.asarray(theta, dtype=np.float64)
    p, o = {}, 0
    for name, shape in layout(rounds):
        k = int(np.prod(shape))
        p[name] = theta[o:o + k].reshape(shape)
        o += k
    assert o == theta.size
    return p


def pack(p, rounds=ROUNDS):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in layout(rounds)])


def init_params(seed, rounds=ROUNDS):
    """Uniform(±1/√fan_in) weights, zero biases; the output layer starts at softplus = 1."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in layout(rounds):
        if name.startswith("W") or name == "w_h2":
            fan_in = shape[0]
            p[name] = rng.uniform(-1.0, 1.0, shape) / np.sqrt(fan_in)
        else:
            p[name] = np.zeros(shape)
    p["w_h2"] = np.zeros(H)
    p["b_h2"] = np.array([INIT_BIAS])
    return pack(p, rounds)


def graph(Ab):
    """Normalised aggregation operators Â (m×n) and Ǎ (n×m) of the scaled constraint matrix."""
    Aabs = abs(sp.csr_matrix(Ab)).tocsr()
    rs = np.asarray(Aabs.sum(axis=1)).ravel()
    cs = np.asarray(Aabs.sum(axis=0)).ravel()
    rinv = np.divide(1.0, rs, out=np.zeros_like(rs), where=rs > 0)
    cinv = np.divide(1.0, cs, out=np.zeros_like(cs), where=cs > 0)
    Ahat = (sp.diags(rinv) @ Aabs).tocsr()
    Acheck = (sp.diags(cinv) @ Aabs.T).tocsr()
    return Ahat, Acheck


def features(Pb, Ab, sigma, l, u):
    """Padded node features (n×32, m×32), ρ̄-independent."""
    Ab = sp.csr_matrix(Ab)
    n, m = Ab.shape[1], Ab.shape[0]
    dP = sp.csr_matrix(Pb).diagonal()
    A2 = Ab.multiply(Ab)
    colsq = np.asarray(A2.sum(axis=0)).ravel()
    rowsq = np.asarray(A2.sum(axis=1)).ravel()
    Aabs = abs(Ab)
    degc = np.diff(sp.csc_matrix(Ab).indptr)
    degr = np.diff(Ab.indptr)
    maxc = np.asarray(Aabs.max(axis=0).todense()).ravel() if Ab.nnz else np.zeros(n)
    maxr = np.asarray(Aabs.max(axis=1).todense()).ravel() if Ab.nnz else np.zeros(m)
    fv = np.zeros((n, 32))
    fv[:, 0] = np.log(dP + sigma)
    fv[:, 1] = np.log(colsq + 1e-12)
    fv[:, 2] = np.log1p(degc)
    fv[:, 3] = np.log(maxc + 1e-12)
    fc = np.zeros((m, 32))
    fc[:, 0] = np.log(rowsq + 1e-12)
    fc[:, 1] = np.log1p(degr)
    fc[:, 2] = (np.asarray(l) == np.asarray(u)).astype(np.float64)
    fc[:, 3] = np.log(maxr + 1e-12)
    return fv, fc, dP, colsq


def head_inputs(dP, colsq, sigma, rho):
    K = dP + sigma + rho * colsq
    phi = np.zeros((dP.size, 32))
    phi[:, 0] = np.log(rho * colsq + 1e-12) - np.log(K)
    phi[:, 1] = np.log(dP + sigma) - np.log(K)
    return phi, K


def relu(x):
    return np.maximum(x, 0.0)


def softplus(g):
    return np.logaddexp(0.0, g)


def sigmoid(g):
    # exp(−log(1 + e^{−g})): exact for very negative g (the tanh form rounds to 0 below g ≈ −37)
    return np.exp(-np.logaddexp(0.0, -g))


def forward(theta, fv, fc, Ahat, Acheck, phi, rounds=ROUNDS):
    p = unpack(theta, rounds)
    c = {}
    hv = relu(fv @ p["W_v0"] + p["b_v0"])
    hc = relu(fc @ p["W_c0"] + p["b_c0"])
    c["hv0"], c["hc0"] = hv, hc
    for l in range(1, rounds + 1):
        ac = Ahat @ hv
        hc = relu(np.hstack([hc, ac]) @ p[f"W_c{l}"] + p[f"b_c{l}"])
        av = Acheck @ hc
        hv = relu(np.hstack([hv, av]) @ p[f"W_v{l}"] + p[f"b_v{l}"])
        c[f"ac{l}"], c[f"hc{l}"], c[f"av{l}"], c[f"hv{l}"] = ac, hc, av, hv
    uh = relu(np.hstack([hv, phi]) @ p["W_h1"] + p["b_h1"])
    g = uh @ p["w_h2"] + p["b_h2"][0]
    c["uh"], c["g"] = uh, g
    return g, c


def loss_and_dg(g, target):
    """L = mean (e − ē)², e = log softplus(g) − target; returns (L, dL/dg)."""
    s = softplus(g)
    e = np.log(s) - target
    d = e - e.mean()
    n = g.size
    L = float(np.mean(d * d))
    dg = (2.0 / n) * d * sigmoid(g) / s
    return L, dg


def backward(theta, fv, fc, Ahat, Acheck, phi, cache, dg, rounds=ROUNDS):
    """Gradient of Σ_i dg_i g_i with respect to the flat parameters (manual chain rule)."""
    p = unpack(theta, rounds)
    G = {k: np.zeros_like(v) for k, v in p.items()}
    uh = cache["uh"]
    hvL = cache[f"hv{rounds}"]
    G["w_h2"] = uh.T @ dg
    G["b_h2"] = np.array([dg.sum()])
    dz = np.outer(dg, p["w_h2"]) * (uh > 0)
    xin = np.hstack([hvL, phi])
    G["W_h1"] = xin.T @ dz
    G["b_h1"] = dz.sum(axis=0)
    dhv = (dz @ p["W_h1"].T)[:, :H]
    dhc = np.zeros_like(cache[f"hc{rounds}"])
    for l in range(rounds, 0, -1):
        hv_prev = cache[f"hv{l - 1}"]
        hc_prev = cache[f"hc{l - 1}"]
        # h_v^l = relu([h_v^{l−1}, a_v] W_vl + b_vl)
        dz = dhv * (cache[f"hv{l}"] > 0)
        G[f"W_v{l}"] = np.hstack([hv_prev, cache[f"av{l}"]]).T @ dz
        G[f"b_v{l}"] = dz.sum(axis=0)
        dx = dz @ p[f"W_v{l}"].T
        dhv_prev = dx[:, :H]
        dav = dx[:, H:]
        # a_v = Ǎ h_c^l
        dhc = dhc + Acheck.T @ dav
        # h_c^l = relu([h_c^{l−1}, a_c] W_cl + b_cl)
        dz = dhc * (cache[f"hc{l}"] > 0)
        G[f"W_c{l}"] = np.hstack([hc_prev, cache[f"ac{l}"]]).T @ dz
        G[f"b_c{l}"] = dz.sum(axis=0)
        dx = dz @ p[f"W_c{l}"].T
        dhc = dx[:, :H]
        dac = dx[:, H:]
        # a_c = Â h_v^{l−1}
        dhv = dhv_prev + Ahat.T @ dac
    dz = dhv * (cache["hv0"] > 0)
    G["W_v0"] = fv.T @ dz
    G["b_v0"] = dz.sum(axis=0)
    dz = dhc * (cache["hc0"] > 0)
    G["W_c0"] = fc.T @ dz
    G["b_c0"] = dz.sum(axis=0)
    return pack(G, rounds)


def loss_grad(theta, fv, fc, Ahat, Acheck, phi, target, rounds=ROUNDS):
    g, cache = forward(theta, fv, fc, Ahat, Acheck, phi, rounds)
    L, dg = loss_and_dg(g, target)
    return L, backward(theta, fv, fc, Ahat, Acheck, phi, cache, dg, rounds), g


def bf16_round(x):
    """Round float64 → bfloat16 (round to nearest even) → float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)
