"""FP64 numpy reference of the learned right preconditioner (test
infrastructure only: used by the tests, never by the library).

The preconditioner is not part of the paper; it is the learned form of the
right preconditioner M in the Krylov solve of eq. (LS_NS), which FGMRES admits
as any variable map.  Definition (what the GPU kernels implement):

  u = D^-1 r                 node-block Jacobi (D = diagonal blocks of A)
  s = sqrt(mean(u^2))        global scale (1 when u = 0)
  f_i = [u_i / s, m_i]       node features, m = 1 on free dofs, 0 on Dirichlet dofs
  h0 = relu(f W_in + b_in)
  for l = 1..L:  g_i = mean over the graph neighbours j of node i (itself
                 included) of h_j;   h = relu([h, g] W_l + b_l)
  delta = h W_out
  z = u + s (m * delta)

The graph is the block pattern of A (rowptr, col).  A pair (r, e) with
A e = r gives the loss  ||m*(z(r) - e)||^2 / ||m*e||^2.

Parameters are one flat vector in the order W_in [F][H], b_in [H], then for
each layer W_l [2H][H], b_l [H], then W_out [H][bs]  (F = 2 bs).

emulate=True evaluates the same map in the arithmetic of the device kernels
instead of FP64: the operands of every dense product that runs on the
matrix cores (the input and hidden layers forward; the weight gradients and
the hidden layers' input gradients backward) rounded to BF16 (nearest even
on the FP32 bit pattern), activations, neighbour means and gradients stored
in FP32, the output layer in FP32 without BF16, the output combination in
FP64.  The products themselves are summed in FP64 here (FP32 on the
device), so the two agree to the accumulation rounding, not bit for bit.
"""
import numpy as np


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _bf16(x):
    """Round to BF16 (nearest even on the FP32 bit pattern), as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(A, B, emulate):
    """A product on the matrix cores: BF16 operands when emulating."""
    return _bf16(A) @ _bf16(B) if emulate else A @ B


def layout(bs, H, L):
    F = 2 * bs
    shapes = [("W_in", (F, H)), ("b_in", (H,))]
    for l in range(L):
        shapes += [(f"W_{l + 1}", (2 * H, H)), (f"b_{l + 1}", (H,))]
    shapes += [("W_out", (H, bs))]
    return shapes


def n_params(bs, H, L):
    return sum(int(np.prod(s)) for _, s in layout(bs, H, L))


def unpack(theta, bs, H, L):
    out, o = {}, 0
    for name, shp in layout(bs, H, L):
        n = int(np.prod(shp))
        out[name] = np.array(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(P, bs, H, L):
    return np.concatenate([P[name].ravel() for name, _ in layout(bs, H, L)])


def block_inverses(rowptr, col, J):
    """Inverse of every diagonal block of the BSR matrix J [nnzb][bs][bs]."""
    N = rowptr.shape[0] - 1
    D = np.zeros((N, J.shape[1], J.shape[2]))
    for i in range(N):
        k = rowptr[i] + int(np.nonzero(col[rowptr[i]:rowptr[i + 1]] == i)[0][0])
        D[i] = np.linalg.inv(J[k])
    return D


def mean_agg(rowptr, col, h):
    N = rowptr.shape[0] - 1
    deg = np.diff(rowptr).astype(np.float64)
    s = np.zeros_like(h)
    rows = np.repeat(np.arange(N), np.diff(rowptr))
    np.add.at(s, rows, h[col])
    return s / deg[:, None]


def mean_agg_T(rowptr, col, y):
    """Transpose of mean_agg: (A^T y)_j = sum over rows i containing j of y_i / deg_i."""
    N = rowptr.shape[0] - 1
    deg = np.diff(rowptr).astype(np.float64)
    rows = np.repeat(np.arange(N), np.diff(rowptr))
    out = np.zeros_like(y)
    np.add.at(out, col, (y / deg[:, None])[rows])
    return out


def forward(theta, rowptr, col, Dinv, mask, r, bs, H, L, keep=False, emulate=False):
    P = unpack(theta, bs, H, L)
    N = rowptr.shape[0] - 1
    st = _f32 if emulate else (lambda x: x)   # storage of the device's FP32 arrays
    r = np.asarray(r, dtype=np.float64).reshape(N, bs)
    u = np.einsum("nij,nj->ni", Dinv, r)
    s = float(np.sqrt(np.mean(u * u)))
    if s == 0.0:
        s = 1.0
    f = st(np.concatenate([u / s, mask], axis=1))
    pre0 = st(_mm(f, P["W_in"], emulate) + P["b_in"])
    h = np.maximum(pre0, 0.0)
    cache = dict(f=f, pre=[pre0], h=[h], g=[], u=u, s=s)
    for l in range(L):
        g = st(mean_agg(rowptr, col, h))
        pre = st(_mm(np.concatenate([h, g], axis=1), P[f"W_{l + 1}"], emulate) + P[f"b_{l + 1}"])
        h = np.maximum(pre, 0.0)
        cache["g"].append(g)
        cache["pre"].append(pre)
        cache["h"].append(h)
    delta = st(h @ P["W_out"])
    z = u + s * (mask * delta)
    return (z, cache) if keep else z


def loss_and_grad(theta, rowptr, col, Dinv, mask, r, e, bs, H, L, emulate=False):
    """Loss of one pair and its gradient with respect to theta (backward pass
    written out layer by layer)."""
    P = unpack(theta, bs, H, L)
    N = rowptr.shape[0] - 1
    st = _f32 if emulate else (lambda x: x)
    e = np.asarray(e, dtype=np.float64).reshape(N, bs)
    if emulate:   # the pair's target is held in FP32
        e = _f32(e)
    z, c = forward(theta, rowptr, col, Dinv, mask, r, bs, H, L, keep=True, emulate=emulate)
    E = float(np.sum((mask * e) ** 2))
    if E == 0.0:
        E = 1.0
    res = mask * (z - e)
    loss = float(np.sum(res * res)) / E
    dz = 2.0 * res / E
    ddelta = st(c["s"] * mask * dz)
    G = {}
    hL = c["h"][-1]
    G["W_out"] = _mm(hL.T, ddelta, emulate)
    dh = st(ddelta @ P["W_out"].T)
    for l in range(L - 1, -1, -1):
        dpre = dh * (c["pre"][l + 1] > 0.0)
        X = np.concatenate([c["h"][l], c["g"][l]], axis=1)
        G[f"W_{l + 1}"] = _mm(X.T, dpre, emulate)
        G[f"b_{l + 1}"] = dpre.sum(axis=0)
        dX = st(_mm(dpre, P[f"W_{l + 1}"].T, emulate))
        dh = st(dX[:, :H] + mean_agg_T(rowptr, col, dX[:, H:]))
    dpre0 = dh * (c["pre"][0] > 0.0)
    G["W_in"] = _mm(c["f"].T, dpre0, emulate)
    G["b_in"] = dpre0.sum(axis=0)
    return loss, pack(G, bs, H, L)
