"""Learned boundary closure: training-data generation, training and export.

Marshalling over include/lbm_closure.h -- the sampling, normalisation,
forward/backward passes, Adam updates and the closure inside the edge kernel
all run in liblbm.so.  PyTorch supplies device memory, streams and the
host-side bookkeeping (site lists, minibatch order).

Training data (row a13 of the design): every member of an ensemble of
uneven pulse/vortex lattices is run inside a twin lattice twice as large per
side, the member's domain centred in it.  At a logged step the inputs of the
member's boundary nodes (every ``stride``-th node of each edge, corners
excluded) are sampled from the twin, where those nodes are interior and see no
boundary; after one step the twin's moments at the same nodes are the
targets, stored as residuals of NSBC's m_c.  Acoustic members are logged only
while nothing reflected at the twin's own boundary can have come back.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import lbm as L

NPARAM = L.LBM_MLP_NPARAM
IN, HID, OUT = 96, 64, 3
CS = 1.0 / math.sqrt(3.0)


def pack_params(p: dict) -> np.ndarray:
    """dict(W1 [64,96], b1, W2 [64,64], b2, W3 [3,64], b3) -> packed fp32 vector."""
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unpack_params(v) -> dict:
    v = np.asarray(v, np.float64)
    out, o = {}, 0
    for k, shp in (("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)),
                   ("b3", (OUT,))):
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp)
        o += n
    return out


def xavier_params(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)

    def xv(n_out, n_in):
        a = math.sqrt(6.0 / (n_in + n_out))
        return rng.uniform(-a, a, size=(n_out, n_in))

    return pack_params({"W1": xv(HID, IN), "b1": np.zeros(HID), "W2": xv(HID, HID), "b2": np.zeros(HID),
                        "W3": xv(OUT, HID) * 0.1, "b3": np.zeros(OUT)})


class Trainer:
    """The library's closure-network trainer on one GPU stream."""

    def __init__(self, params=None, max_batch=4096, device="cuda", seed=0):
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.max_batch = int(max_batch)
        p = xavier_params(seed) if params is None else np.asarray(params, np.float32)
        assert p.size == NPARAM
        self._p0 = torch.from_numpy(p.astype(np.float32)).to(self.device)
        nbytes = L.lbm_mlp_workspace_bytes(self.max_batch)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.m = L.lbm_mlp_init(self.max_batch, self.workspace.data_ptr(), nbytes, self._p0.data_ptr(),
                                self.stream.cuda_stream)
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def fit_normalization(self, feat: torch.Tensor, resid: torch.Tensor):
        L.lbm_mlp_fit_normalization(self.m, feat.data_ptr(), resid.data_ptr(), feat.shape[0])

    def normalization(self):
        mean = torch.zeros(96, device=self.device)
        inv = torch.zeros(96, device=self.device)
        sc = torch.zeros(3, device=self.device)
        L.lbm_mlp_normalization(self.m, mean.data_ptr(), inv.data_ptr(), sc.data_ptr())
        self.stream.synchronize()
        return mean.cpu().numpy(), inv.cpu().numpy(), sc.cpu().numpy()

    def pack(self, feat: torch.Tensor, resid: torch.Tensor | None = None):
        n = feat.shape[0]
        x = torch.empty((n, IN), dtype=torch.bfloat16, device=self.device)
        t = torch.empty((n, OUT), dtype=torch.float32, device=self.device) if resid is not None else None
        L.lbm_mlp_pack(self.m, feat.data_ptr(), resid.data_ptr() if resid is not None else None, n, x.data_ptr(),
                       t.data_ptr() if t is not None else None)
        return x, t

    def train_step(self, x, t, lr, rows=None, batch=None):
        batch = int(batch if batch is not None else (rows.numel() if rows is not None else x.shape[0]))
        L.lbm_mlp_train_step(self.m, x.data_ptr(), t.data_ptr(), x.shape[0],
                             rows.data_ptr() if rows is not None else None, batch, lr, self._loss.data_ptr())
        return self._loss

    def grads(self, x, t, rows=None, batch=None):
        batch = int(batch if batch is not None else (rows.numel() if rows is not None else x.shape[0]))
        g = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        L.lbm_mlp_grads(self.m, x.data_ptr(), t.data_ptr(), x.shape[0], rows.data_ptr() if rows is not None else None,
                        batch, g.data_ptr(), self._loss.data_ptr())
        self.stream.synchronize()
        return g.cpu().numpy(), float(self._loss.item())

    def forward(self, x):
        y = torch.empty((x.shape[0], OUT), dtype=torch.float32, device=self.device)
        L.lbm_mlp_forward(self.m, x.data_ptr(), x.shape[0], y.data_ptr())
        return y

    def params(self) -> np.ndarray:
        out = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        L.lbm_mlp_params(self.m, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy()

    def export(self, trust: float = 6.0) -> torch.Tensor:
        blob = torch.empty(L.lbm_closure_net_bytes(), dtype=torch.uint8, device=self.device)
        L.lbm_mlp_export(self.m, trust, blob.data_ptr())
        return blob

    def train(self, x, t, epochs=20, batch=4096, lr=2e-3, lr_end=2e-4, seed=0, log=None):
        """Shuffled minibatch Adam with a geometric learning-rate decay; returns per-epoch mean losses."""
        n = x.shape[0]
        g = torch.Generator().manual_seed(seed)
        nb = max(1, n // batch)
        total = epochs * nb
        losses = []
        k = 0
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g)[: nb * batch].to(torch.int32).to(self.device)
            acc = torch.zeros((), device=self.device)
            for b in range(nb):
                lr_k = lr * (lr_end / lr) ** (k / max(1, total - 1))
                acc += self.train_step(x, t, lr_k, rows=perm[b * batch:(b + 1) * batch])[0]
                k += 1
            losses.append(float(acc.item()) / nb)
            if log:
                log(f"epoch {ep}: loss {losses[-1]:.5f}")
        return losses

    def close(self):
        if getattr(self, "m", None) is not None:
            L.lbm_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ sites and data

def edge_sites(nx, ny, stride=1, x0=0, y0=0, margin=1):
    """Boundary nodes of an nx x ny window whose lower-left node is (x0, y0) in some lattice:
    rows (x, y, edge) for every ``stride``-th node of each edge, ``margin`` nodes kept away
    from the corners.  edge = 0 left, 1 right, 2 bottom, 3 top (outward normal)."""
    out = []
    for y in range(margin, ny - margin, stride):
        out.append((x0, y0 + y, 0))
        out.append((x0 + nx - 1, y0 + y, 1))
    for x in range(margin, nx - margin, stride):
        out.append((x0 + x, y0, 2))
        out.append((x0 + x, y0 + ny - 1, 3))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def twin_fields(member_fields_fn, m, pad_x, pad_y):
    """Fields of the twin of ensemble member m: the member's analytic field on a lattice padded by
    (pad_x, pad_y) on each side (the member's node (0, 0) at twin node (pad_x, pad_y))."""
    return member_fields_fn(m, offset=(pad_x, pad_y), nx=m.nx + 2 * pad_x, ny=m.ny + 2 * pad_y)


def generate_dataset(members, member_fields_fn, member_m0_fn, steps=2000, log_every=10, stride=4, store="f32",
                     gamma=0.6, device="cuda", log=None):
    """Run the twins of `members` as one ensemble and collect (raw inputs, residual targets).

    Returns (feat [M, 96] float32, resid [M, 3] float32) device tensors."""
    from .ensemble import Ensemble, member_params
    twins, fields, sites, t_clean = [], [], [], []
    for k, m in enumerate(members):
        px, py = m.nx // 2, m.ny // 2
        u0 = member_m0_fn(m)[1:]
        twins.append(member_params(m.nx + 2 * px, m.ny + 2 * py, m.tau, store=store, gamma=gamma,
                                   ubase=u0 if m.kind == "vortex" else (0.0, 0.0)))
        fields.append(twin_fields(member_fields_fn, m, px, py))
        s = edge_sites(m.nx, m.ny, stride, px, py)
        sites.append(np.concatenate([np.full((len(s), 1), k, np.int32), s, np.zeros((len(s), 1), np.int32)], 1)[:, :4])
        speed = CS + math.hypot(*u0)
        t_clean.append(math.inf if m.kind == "vortex" else 1.25 * min(m.nx, m.ny) / speed)
    ens = Ensemble(twins, fields, device=device)
    for k, m in enumerate(members):
        ens.set_farfield(k, 0.0, *member_m0_fn(m))
    feats, resids = [], []
    t = 0
    while t + 1 <= steps:
        live = np.concatenate([s for s, tc in zip(sites, t_clean) if t + 1 <= tc])
        if len(live):
            sd = torch.from_numpy(np.ascontiguousarray(live)).to(device)
            n = len(live)
            f = torch.empty((n, IN), dtype=torch.float32, device=device)
            mc = torch.empty((n, OUT), dtype=torch.float32, device=device)
            L.lbm_ens_closure_features(ens.ens, sd.data_ptr(), n, f.data_ptr(), mc.data_ptr())
            ens.step(1)
            r = torch.empty((n, OUT), dtype=torch.float32, device=device)
            L.lbm_ens_closure_moments(ens.ens, sd.data_ptr(), n, mc.data_ptr(), r.data_ptr())
            feats.append(f)
            resids.append(r)
            adv = 1
        else:
            adv = 0
        rest = min(log_every - adv, steps - t - adv)
        if rest > 0:
            ens.step_graph(rest)
        t += adv + max(rest, 0)
        if log and len(feats) % 20 == 1:
            log(f"t={t} samples={sum(x.shape[0] for x in feats)}")
    ens.close()
    feat = torch.cat(feats)
    resid = torch.cat(resids)
    ok = torch.isfinite(feat).all(1) & torch.isfinite(resid).all(1)
    return feat[ok].contiguous(), resid[ok].contiguous()
