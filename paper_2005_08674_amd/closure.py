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

    def set_normalization(self, mean, inv_std, scale):
        t = [torch.as_tensor(np.asarray(v, np.float32)).to(self.device) for v in (mean, inv_std, scale)]
        L.lbm_mlp_set_normalization(self.m, t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr())
        self.stream.synchronize()

    def save(self, path, **meta):
        """Parameters and normalisation (+ `meta` scalars such as trust and gain) as .npz."""
        mean, inv, sc = self.normalization()
        np.savez(path, params=self.params(), feat_mean=mean, feat_inv_std=inv, out_scale=sc,
                 **{k: np.float64(v) for k, v in meta.items()})

    @classmethod
    def load(cls, path, max_batch=4096, device="cuda"):
        d = np.load(path)
        tr = cls(d["params"], max_batch=max_batch, device=device)
        tr.set_normalization(d["feat_mean"], d["feat_inv_std"], d["out_scale"])
        tr.meta = {k: float(d[k]) for k in d.files if d[k].ndim == 0}
        return tr

    def export(self, trust: float = None, gain: float = None, kmin: float = None) -> torch.Tensor:
        """Network blob for lbm_set_closure; trust, gain and the regime gate kmin default to the
        values saved with the network (else 1.0, 1.0 and 0.0)."""
        meta = getattr(self, "meta", {})
        trust = meta.get("trust", 1.0) if trust is None else trust
        gain = meta.get("gain", 1.0) if gain is None else gain
        kmin = meta.get("kmin", 0.0) if kmin is None else kmin
        blob = torch.empty(L.lbm_closure_net_bytes(), dtype=torch.uint8, device=self.device)
        L.lbm_mlp_export(self.m, trust, gain, kmin, blob.data_ptr())
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


def kinetic_ratio(feat: torch.Tensor, rho0: float = 1.0) -> torch.Tensor:
    """Per input row, the strip's kinetic disturbance sum |u - u_ref|^2 over its acoustic part
    sum c_s^2 (rho - rho_ref)^2 / rho0^2 (the quantity the regime gate kmin thresholds)."""
    s = feat[:, :81].reshape(-1, 9, 9)
    su = (s[:, :, 1] ** 2 + s[:, :, 2] ** 2).sum(1)
    sr = (s[:, :, 0] ** 2).sum(1) / (3.0 * rho0 * rho0)
    return su / sr


def clean_time(m, u0, pad_x, pad_y, core=4.0):
    """Last time at which the twin of member m (padded pad_x, pad_y per side) still gives clean targets
    at the member's boundary nodes, i.e. before anything its own boundary did can have reached them.
    - Pulse (acoustic) members: the sound from the disturbance, moving at c_s + |u0|, reaches the twin's
      edge and comes back: 1.25 min(nx, ny) / (c_s + |u0|) (the twin edge lies N/2 beyond the member's).
    - Vortex members: the swirl (significant within `core` core radii of the centre: 4 r_c leaves
      1e-3 of its peak) is carried at u0 from (xc, yc); once it touches the twin's edge, the edge's
      response needs min(pad_x, pad_y) / (c_s + |u0|) more steps to reach the member's boundary.
      The acoustic transient of the vortex's initial state is left out of this bound.
    The member's node (0, 0) is the twin's node (pad_x, pad_y)."""
    speed = CS + math.hypot(*u0)
    if m.kind != "vortex":
        return 1.25 * min(m.nx, m.ny) / speed
    p = m.params
    rd = core * p["rc"]
    t_touch = math.inf
    for c, v, n, pad in ((p["xc"], u0[0], m.nx, pad_x), (p["yc"], u0[1], m.ny, pad_y)):
        if v > 0:
            t_touch = min(t_touch, max(0.0, (n - 1 + pad) - (c + rd)) / v)
        elif v < 0:
            t_touch = min(t_touch, max(0.0, (c - rd) - (-pad)) / -v)
    return t_touch + min(pad_x, pad_y) / speed


def generate_dataset(members, member_fields_fn, member_m0_fn, steps=2000, log_every=10, stride=4, store="f32",
                     gamma=0.6, net=None, amp_min=1e-8, amp_rel=0.0, kmin=0.0, device="cuda", log=None):
    """Run every member (NSBC edges, or the closure `net` with NSBC fallback) beside its twin in one
    ensemble and collect (raw inputs, residual targets).

    Inputs come from the member's own boundary nodes, so they carry what the boundary condition in
    use did at earlier steps; targets are the twin's moments at the same physical nodes one step
    later, minus the member's NSBC prediction m_c, divided by the strip amplitude A.  The whole run is
    one graph launch that logs every site every `log_every` steps (lbm_ens_step_graph); a record is
    kept for a member only while the twin is clean there (clean_time).  Sites whose A is at most
    `amp_min` (no disturbance yet, only rounding noise) or below `amp_rel` times the largest A logged
    on the same member are left out, and so are sites outside the regime gate (kinetic_ratio <=
    kmin).  Returns (feat [M, 96], resid [M, 3]) float32 device tensors."""
    from .ensemble import Ensemble, member_params
    count = len(members)
    lat, fields, msites, tsites, t_clean, m0s = [], [], [], [], [], []
    for k, m in enumerate(members):
        u0 = tuple(member_m0_fn(m)[1:])
        ub = u0 if m.kind == "vortex" else (0.0, 0.0)
        lat.append(member_params(m.nx, m.ny, m.tau, store=store, gamma=gamma, ubase=ub))
        fields.append(member_fields_fn(m))
        s = edge_sites(m.nx, m.ny, stride)
        msites.append(np.concatenate([np.full((len(s), 1), k, np.int32), s], 1))
        m0s.append(member_m0_fn(m))
        t_clean.append(clean_time(m, u0, m.nx // 2, m.ny // 2))
    for k, m in enumerate(members):
        px, py = m.nx // 2, m.ny // 2
        u0 = tuple(member_m0_fn(m)[1:])
        ub = u0 if m.kind == "vortex" else (0.0, 0.0)
        lat.append(member_params(m.nx + 2 * px, m.ny + 2 * py, m.tau, store=store, gamma=gamma, ubase=ub))
        fields.append(twin_fields(member_fields_fn, m, px, py))
        s = msites[k].copy()
        s[:, 0] = count + k
        s[:, 1] += px
        s[:, 2] += py
        tsites.append(s)
    ens = Ensemble(lat, fields, device=device)
    for k in range(count):
        ens.set_farfield(k, 0.0, *m0s[k])
        ens.set_farfield(count + k, 0.0, *m0s[k])
    if net is not None:
        for k in range(count):
            L.lbm_ens_set_closure(ens.ens, k, net.data_ptr(), 1)
    ms = torch.from_numpy(np.ascontiguousarray(np.concatenate(msites))).to(device)
    ts = torch.from_numpy(np.ascontiguousarray(np.concatenate(tsites))).to(device)
    ens.set_log_sites(ms, ts)
    f, mc, r = ens.step_graph_logged(steps, log_every)
    ens.close()
    # record j holds step t_j = j * log_every; keep a member's rows while t_j + 1 <= its clean time
    tc = torch.tensor(t_clean, dtype=torch.float64, device=device)[ms[:, 0].long()]
    tj = torch.arange(f.shape[0], dtype=torch.float64, device=device)[:, None] * log_every
    keep = (tj + 1 <= tc[None, :]) & (mc[:, :, OUT] > amp_min)
    feats, resids, amps = [f[keep]], [r[keep]], [mc[:, :, OUT][keep]]
    mids = [ms[:, 0].long()[None, :].expand(f.shape[0], -1)[keep]]
    if log:
        log(f"{f.shape[0]} records of {f.shape[1]} sites, {int(keep.sum())} kept")
    feat = torch.cat(feats)
    resid = torch.cat(resids)
    ok = torch.isfinite(feat).all(1) & torch.isfinite(resid).all(1)
    if kmin > 0.0:
        ok &= kinetic_ratio(feat) > kmin
    if amp_rel > 0.0:
        amp, mid = torch.cat(amps), torch.cat(mids)
        top = torch.zeros(count, dtype=amp.dtype, device=device).scatter_reduce(
            0, mid[ok], amp[ok], reduce="amax", include_self=True)
        ok &= amp >= amp_rel * top[mid]
    return feat[ok].contiguous(), resid[ok].contiguous()


def heldout_mse(trainer: "Trainer", x, t, chunk=None):
    """Mean squared error of the trained network on packed samples (library loss kernel, no update)."""
    chunk = chunk or trainer.max_batch
    tot, n = 0.0, x.shape[0]
    for s in range(0, n, chunk):
        b = min(chunk, n - s)
        _, loss = trainer.grads(x[s:s + b], t[s:s + b])
        tot += loss * b
    return tot / n


def main(argv=None):
    """Train the closure on the batched-ensemble members and their twins and report its one-step gain
    on held-out members."""
    import argparse
    import json
    import sys
    import time
    from . import workloads as W

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--log-every", type=int, default=10)
    ap.add_argument("--stride", type=int, default=4)
    ap.add_argument("--amp-rel", type=float, default=0.1,
                    help="keep sites whose strip amplitude is at least this fraction of the member's largest")
    ap.add_argument("--epochs", type=int, default=15)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-end", type=float, default=1e-4)
    ap.add_argument("--heldout-members", type=int, default=32)
    ap.add_argument("--heldout-seed", type=int, default=40)
    ap.add_argument("--rounds", type=int, default=1, help="data rounds; rounds >= 1 run the members with the "
                                                           "previous round's network")
    ap.add_argument("--trust", type=float, default=1.0, help="trust bound saved with the network")
    ap.add_argument("--gain", type=float, default=1.0, help="correction gain saved with the network")
    ap.add_argument("--kmin", type=float, default=10.0,
                    help="regime gate saved with the network: the correction applies where the strip's kinetic "
                         "disturbance exceeds kmin times its acoustic part (0: everywhere)")
    ap.add_argument("--train-kmin", type=float, default=0.0,
                    help="train only on sites above this kinetic/acoustic ratio (0: every regime)")
    ap.add_argument("--out", default=None, help="save params + normalisation (.npz)")
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    def data(members, net=None):
        return generate_dataset(members, W.member_fields, W.member_m0, steps=args.steps, log_every=args.log_every,
                                stride=args.stride, amp_rel=args.amp_rel, kmin=args.train_kmin, net=net)

    t0 = time.time()
    members = W.ensemble_members(args.members, seed=args.seed)
    feat, resid = data(members)
    t_data = time.time() - t0
    log(f"dataset round 0 (NSBC edges): {feat.shape[0]} samples in {t_data:.1f} s")
    tr = Trainer(max_batch=args.batch)
    tr.fit_normalization(feat, resid)
    x, t = tr.pack(feat, resid)
    t1 = time.time()
    losses = tr.train(x, t, epochs=args.epochs, batch=args.batch, lr=args.lr, lr_end=args.lr_end, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    for rnd in range(1, args.rounds):
        # closed-loop data: the members now run with the current network on their edges
        f2, r2 = data(members, net=tr.export(args.trust, args.gain, args.kmin))
        log(f"dataset round {rnd} (closure edges): {f2.shape[0]} samples")
        feat, resid = torch.cat([feat, f2]), torch.cat([resid, r2])
        del f2, r2
        x, t = tr.pack(feat, resid)
        t1 = time.time()
        losses = tr.train(x, t, epochs=args.epochs, batch=args.batch, lr=args.lr, lr_end=args.lr_end,
                          seed=rnd, log=log)
        torch.cuda.synchronize()
        t_train += time.time() - t1
    del feat, resid
    ho = W.ensemble_members(args.heldout_members, seed=args.heldout_seed)
    hf, hr = data(ho)
    hx, ht = tr.pack(hf, hr)
    mse_net = heldout_mse(tr, hx, ht)
    mse_nsbc = float((ht.double() ** 2).mean().item())  # NSBC predicts a zero residual
    if args.out:
        tr.save(args.out, trust=args.trust, gain=args.gain, kmin=args.kmin)
    res = {"train_samples": int(x.shape[0]), "heldout_samples": int(hx.shape[0]), "epochs": args.epochs,
           "first_loss": losses[0], "final_loss": losses[-1], "heldout_mse_closure": mse_net,
           "heldout_mse_nsbc": mse_nsbc, "heldout_gain": 1.0 - mse_net / mse_nsbc,
           "data_s": round(t_data, 2), "train_s": round(t_train, 2),
           "train_steps": args.epochs * (x.shape[0] // args.batch)}
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
