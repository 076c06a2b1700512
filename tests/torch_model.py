"""Test-only float64 PyTorch restatement of the model for tiny molecules.

It pins the oracle's hand-derived gradient against PyTorch autograd.  It is
written independently of the oracle (dense all-pairs tensors, the angular
term through acos rather than the sqrt identity) and is never used by the
product path.
"""

import math

import torch

ETA_R, RC_R = 16.0, 5.2
ETA_A, RC_A, ZETA = 8.0, 3.5, 32.0
RADIAL = torch.linspace(0.9, 5.1, 16, dtype=torch.float64)
SHELLS = torch.tensor([0.9, 1.55, 2.2, 2.85], dtype=torch.float64)
SECTORS = (2 * torch.arange(8, dtype=torch.float64) + 1) * math.pi / 16
PAIR = [[0, 1, 2, 3], [1, 4, 5, 6], [2, 5, 7, 8], [3, 6, 8, 9]]
SHAPES = ((160, 384), (128, 160), (96, 128), (1, 96))


def unpack(weights):
    w = torch.as_tensor(weights).to(torch.float64)
    per = sum(o * i + o for o, i in SHAPES)
    out = []
    for e in range(4):
        off = e * per
        layers = []
        for (o, i) in SHAPES:
            W = w[off:off + o * i].reshape(o, i)
            off += o * i
            b = w[off:off + o]
            off += o
            layers.append((W, b))
        out.append(layers)
    return out


def fc(r, rc):
    return torch.where(r < rc, 0.5 * torch.cos(math.pi * r / rc) + 0.5, torch.zeros_like(r))


def descriptors(pos, species):
    n = pos.shape[0]
    d = pos[None, :, :] - pos[:, None, :]                  # d[i, j] = x_j - x_i
    eye = torch.eye(n, dtype=torch.bool)
    r = torch.sqrt((d * d).sum(-1) + eye.to(pos.dtype))     # avoid sqrt(0) on the diagonal
    G = torch.zeros(n, 384, dtype=pos.dtype)
    onehot = torch.nn.functional.one_hot(torch.as_tensor(species).long(), 4).to(pos.dtype)
    rad = torch.exp(-ETA_R * (r[..., None] - RADIAL) ** 2) * fc(r, RC_R)[..., None]
    rad = rad * (~eye)[..., None]
    G[:, :64] = torch.einsum("ijk,js->isk", rad, onehot).reshape(n, 64)
    for i in range(n):
        for j in range(n):
            for k in range(j + 1, n):
                if i in (j, k) or not (r[i, j] < RC_A and r[i, k] < RC_A):
                    continue
                cos = (d[i, j] * d[i, k]).sum() / (r[i, j] * r[i, k])
                theta = torch.acos(0.95 * cos)
                A = (1 + torch.cos(theta - SECTORS)) ** ZETA
                B = torch.exp(-ETA_A * ((r[i, j] + r[i, k]) / 2 - SHELLS) ** 2)
                w = 2.0 ** (1 - ZETA) * fc(r[i, j], RC_A) * fc(r[i, k], RC_A)
                p = PAIR[int(species[j])][int(species[k])]
                G[i, 64 + 32 * p:64 + 32 * p + 32] = G[i, 64 + 32 * p:64 + 32 * p + 32] + \
                    (w * B[:, None] * A[None, :]).reshape(32)
    return G


def network(layers, x):
    for li, (W, b) in enumerate(layers):
        x = torch.nn.functional.linear(x, W, b)
        if li < 3:
            # CELU written with exp so that autograd differentiates exp itself
            # (torch's fused CELU backward loses accuracy for very negative z)
            neg = 0.1 * (torch.exp(torch.clamp(x, max=0.0) / 0.1) - 1.0)
            x = torch.where(x > 0, x, neg)
    return x.squeeze(-1)


def energy_forces(pos, species, weights):
    nets = unpack(weights)
    x = torch.tensor(pos, dtype=torch.float64, requires_grad=True)
    G = descriptors(x, species)
    E = torch.zeros((), dtype=torch.float64)
    for e in range(4):
        m = torch.as_tensor(species) == e
        if m.any():
            E = E + network(nets[e], G[m]).sum()
    (g,) = torch.autograd.grad(E, x)
    return float(E), (-g).numpy()
