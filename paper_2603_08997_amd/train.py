"""Post-densification training loop with the SkipGS backward gate, driven
through the C ABI. Per iteration (Algorithm 1): sample a view, render it,
compute the loss, update the gate on the device, and, predicated on the
gate's device flag, run the loss backward, the render backward and Adam.
Nothing is read back to the host inside the loop.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import scenes as S
from . import skipgs as sk


@dataclass
class StageTimer:
    """Optional HIP events around each stage of an iteration (on the stream
    the kernels run on)."""
    names: tuple = ("project", "bin", "rasterize", "loss", "gate", "loss_bwd", "raster_bwd",
                    "project_bwd", "adam")
    events: list = field(default_factory=list)

    def mark(self):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def summary(self, mask=None):
        """Mean ms per stage over the recorded iterations (optionally only those in mask)."""
        out = {k: [] for k in self.names}
        for it, evs in enumerate(self.events):
            if mask is not None and not mask[it]:
                continue
            for k, (a, b) in evs.items():
                out[k].append(a.elapsed_time(b))
        return {k: (float(np.mean(v)) if v else 0.0) for k, v in out.items()}

    def per_iter(self, name):
        return np.array([evs[name][0].elapsed_time(evs[name][1]) if name in evs else np.nan
                         for evs in self.events])


class Trainer:
    """Holds the device state of one training run: parameters, Adam moments,
    gradient buffer, gate state, per-view targets, workspaces, the device
    camera table and the device view sequence.

    Two ways to run an iteration, with identical kernels and results:
    ``step()`` enqueues one sgs_train_iteration (the view is read on the
    device from the sequence, so the call can be captured in a graph and
    replayed); ``iteration()`` calls the stages one by one, with optional
    HIP events between them, for the stage breakdown."""

    def __init__(self, init: S.Scene | None, cams, targets: torch.Tensor, rp: sk.RasterParams,
                 gate: sk.GateParams | None, capacity: int, lrs=None, gated: bool = True,
                 fused: bool = True, sequence=None, visible_only: bool = False, device="cuda",
                 state=None):
        """state: (planes, m, v, step_count, n, sh_degree) device tensors to
        continue from (a set produced by densification) instead of ``init``."""
        self.dev = torch.device(device)
        self.cams = list(cams)
        self.rp = rp
        self.cap = int(capacity)
        self.gated = gated
        self.fused = fused
        if state is None:
            self.n = init.n
            self.deg = init.sh_degree
            self.planes = torch.as_tensor(init.to_planes()).to(self.dev)
            self.m = torch.zeros_like(self.planes)
            self.v = torch.zeros_like(self.planes)
            self.step_count = torch.zeros(1, dtype=torch.int32, device=self.dev)
        else:
            self.planes, self.m, self.v, self.step_count, self.n, self.deg = state
        self.grads = torch.zeros_like(self.planes)
        self.adam = sk.AdamParams(lr=lrs or sk.default_lrs(self.deg), visible_only=visible_only)
        self.targets = targets            # [views][3 H W]
        W, H = self.cams[0].width, self.cams[0].height
        assert all(c.width == W and c.height == H for c in self.cams)
        self.W, self.H = W, H
        self.ws = sk.alloc_bytes(sk.forward_workspace_size(rp, self.n, [self.cams[0]], self.cap))
        self.ws.zero_()
        self.lws = sk.alloc_bytes(sk.loss_workspace_size(W, H)).zero_()
        self.rgb = torch.zeros(3 * W * H, device=self.dev)
        self.dl = torch.zeros_like(self.rgb)
        self.loss = torch.zeros(1, device=self.dev)
        self.gate = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.gp = gate
        if gated:
            self.gstate = sk.alloc_bytes(sk.gate_state_size(gate))
            sk.gate_init(gate, self.gstate)
        # device view sequence and the slot the iteration reads its view from
        seq = np.zeros(1, np.int32) if sequence is None else np.asarray(sequence, np.int32)
        self.seq = torch.as_tensor(seq).to(self.dev)
        self.seq_pos = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.view = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.table = sk.camera_table(self.cams, rp)
        self.train_step = sk.TrainStep(
            self.planes, self.n, self.deg, self.cams, self.table, self.view, rp, self.ws, self.cap,
            self.targets, 0.2, self.lws, self.rgb, self.dl, self.loss,
            gate if gated else None, self.gstate if gated else None, self.gate, self.adam, self.m,
            self.v, self.step_count)
        # pre-marshalled arguments for the stage-by-stage path
        self.prep = sk.Prepared(self.planes, self.n, self.deg, self.cams, rp, self.ws, self.cap)
        self.rgb_p, self.dl_p = self.rgb.data_ptr(), self.dl.data_ptr()
        self.lws_p, self.lws_n = self.lws.data_ptr(), self.lws.numel()
        self.planes_p, self.grads_p = self.planes.data_ptr(), self.grads.data_ptr()
        self.m_p, self.v_p = self.m.data_ptr(), self.v.data_ptr()
        self.step_p = self.step_count.data_ptr()
        self.stride, self.F = int(self.planes.shape[1]), int(self.planes.shape[0])
        self.adamc = self.adam.c()
        if gated:
            self.gpc = gate.c()
            self.gstate_p = self.gstate.data_ptr()

    def step(self, stream=None):
        """Enqueue the next iteration of the sequence (two calls, no host
        synchronisation; capturable)."""
        s = torch.cuda.current_stream().cuda_stream if stream is None else stream
        sk._check(sk.LIB.sgs_view_sequence_next(self.seq.data_ptr(), int(self.seq.numel()),
                                                self.seq_pos.data_ptr(), self.view.data_ptr(), s))
        self.train_step(s)

    def iteration(self, view: int, d_view: torch.Tensor, gate_slot: torch.Tensor,
                  loss_slot: torch.Tensor | None = None, timer: StageTimer | None = None):
        """Enqueue one iteration stage by stage. view: the host view index;
        d_view: a device int32[1] holding the same index (the gate reads it);
        gate_slot: a device int32[1] that receives the decision (forced to 1
        in a full run)."""
        P, s = self.prep, torch.cuda.current_stream().cuda_stream
        gate = gate_slot.data_ptr()
        loss = self.loss if loss_slot is None else loss_slot
        lossp = loss.data_ptr()
        tgt = self.targets[view].data_ptr()
        mark = timer.mark if timer is not None else (lambda: None)
        e0 = mark()
        P.project(view, s)
        e1 = mark()
        P.bin(view, s)
        e2 = mark()
        P.rasterize(view, self.rgb_p, s)
        e3 = mark()
        sk._check(sk.LIB.sgs_photometric_loss(self.rgb_p, tgt, self.W, self.H, C.c_float(0.2),
                                              self.lws_p, self.lws_n, lossp, s))
        e4 = mark()
        if self.gated:
            sk._check(sk.LIB.sgs_gate_update(C.byref(self.gpc), self.gstate_p, d_view.data_ptr(),
                                             lossp, gate, s))
        else:
            gate_slot.fill_(1)
        e5 = mark()
        sk._check(sk.LIB.sgs_photometric_loss_backward(self.rgb_p, tgt, self.W, self.H,
                                                       C.c_float(0.2), self.lws_p, self.lws_n,
                                                       gate, self.dl_p, s))
        e6 = mark()
        P.rasterize_backward(view, self.dl_p, gate, s)
        e7 = mark()
        if self.fused:
            # projection backward and Adam in one pass; no gradient array
            P.project_backward_adam(view, self.adamc, self.m_p, self.v_p, self.step_p, gate, s)
            e8 = mark()
        else:
            P.project_backward(view, gate, self.grads_p, s)
            e8 = mark()
            sk._check(sk.LIB.sgs_adam_step(C.byref(self.adamc), self.planes_p, self.grads_p,
                                           self.m_p, self.v_p, self.n, self.stride, self.F,
                                           self.step_p, gate, s))
        e9 = mark()
        if timer is not None:
            es = [e0, e1, e2, e3, e4, e5, e6, e7, e8, e9]
            timer.events.append({k: (es[i], es[i + 1]) for i, k in enumerate(timer.names)})

    def backward_count(self) -> tuple[int, int]:
        """(executed backward passes, iterations) the gate has seen (syncs)."""
        if not self.gated:
            return int(self.step_count.item()), int(self.step_count.item())
        snap = sk.gate_read(self.gp, self.gstate)
        return int(snap["b"]), int(snap["t"])

    def render(self, view: int, out: torch.Tensor):
        self.prep.render_forward(view, out.data_ptr(), torch.cuda.current_stream().cuda_stream)

    def mean_loss(self, views) -> float:
        """Forward-only sweep: mean photometric loss over the given views."""
        vals = torch.zeros(len(views), device=self.dev)
        for i, v in enumerate(views):
            self.render(v, self.rgb)
            sk.photometric_loss(self.rgb, self.targets[v], self.W, self.H, 0.2, self.lws,
                                vals[i:i + 1])
        return float(vals.mean().item())

    def status(self):
        return sk.read_status(self.ws)


def render_targets(gt: S.Scene, cams, rp, capacity, device="cuda") -> torch.Tensor:
    """Ground-truth images of every view, rendered from the ground-truth set."""
    planes = torch.as_tensor(gt.to_planes()).to(device)
    W, H = cams[0].width, cams[0].height
    ws = sk.alloc_bytes(sk.forward_workspace_size(rp, gt.n, [cams[0]], capacity)).zero_()
    out = torch.zeros(len(cams), 3 * W * H, device=device)
    for i, c in enumerate(cams):
        sk.render_forward(planes, gt.n, gt.sh_degree, [c], rp, ws, capacity, out[i])
    flags, _, _ = sk.read_status(ws)
    if flags:
        raise RuntimeError(f"target rendering overflowed pair capacity ({flags})")
    return out


def measure_capacity(scene: S.Scene, cams, rp, device="cuda", probe_capacity=1 << 16) -> int:
    """Largest pair capacity a forward of one view needs over the views (the
    larger of its super-tile pairs and the tile-list entries it records; one
    synchronisation per view). Each view is rendered with a capacity that
    suffices, probing again with the reported need when the first try
    overflows."""
    planes = torch.as_tensor(scene.to_planes()).to(device)
    out = torch.empty(3 * cams[0].width * cams[0].height, device=device)
    cap = int(probe_capacity)
    ws = None
    best = 0
    for c in cams:
        for _ in range(3):
            if ws is None:
                ws = sk.alloc_bytes(sk.forward_workspace_size(rp, scene.n, [c], cap)).zero_()
            sk.clear_status(ws)
            sk.render_forward(planes, scene.n, scene.sh_degree, [c], rp, ws, cap, out)
            flags, _, need = sk.read_status(ws)
            if not flags & sk.STATUS_PAIR_OVERFLOW:
                break
            cap = int(need * 1.25) + 4096
            ws = None
        best = max(best, need)
    del ws, planes, out
    return best


def densify_step(tr: Trainer, dp: sk.DensifyParams, grad_sum: torch.Tensor, count: torch.Tensor,
                 rng: np.random.Generator):
    """One clone / split / prune step of the trainer's set (adaptive density
    control, Sec. 3). Returns (planes, m, v, n) of the new set with a padded
    stride; every Gaussian yields at most two, so the output cannot overflow."""
    n, F = tr.n, tr.F
    normals = torch.as_tensor(rng.standard_normal((max(n, 1), 2, 3)), dtype=torch.float32,
                              device=tr.dev)
    cap = S.padded_stride(max(2 * n, 1))
    outs = [torch.empty(F, cap, device=tr.dev) for _ in range(3)]
    ws = sk.alloc_bytes(sk.densify_workspace_size(n))
    d_n = torch.zeros(1, dtype=torch.int64, device=tr.dev)
    sk.densify(dp, tr.planes, n, tr.deg, tr.m, tr.v, grad_sum, count, normals, *outs, ws, d_n)
    n_new = int(d_n.item())
    stride = S.padded_stride(max(n_new, 1))
    planes, m, v = (torch.zeros(F, stride, device=tr.dev) for _ in range(3))
    for dst, src in zip((planes, m, v), outs):
        dst[:, :n_new] = src[:, :n_new]
    return planes, m, v, n_new


def train_two_phase(init: S.Scene, cams, targets: torch.Tensor, rp: sk.RasterParams,
                    gate: sk.GateParams, dp: sk.DensifyParams, densify_until: int,
                    densify_every: int, post_iters: int, sequence, capacity_per_gaussian: int = 64,
                    seed: int = 0, log=None) -> dict:
    """Two-phase training (Sec. 3): full-backward iterations with the
    view-space gradient statistic gathered after every backward and a clone /
    split / prune step every ``densify_every`` iterations until
    ``densify_until`` (T_d); from then on the set is fixed and the SkipGS gate
    decides every backward (Algorithm 1), starting at t = 1. ``sequence``: the
    view of every iteration (both phases)."""
    rng = np.random.default_rng(seed)
    seq = np.asarray(sequence, np.int64)
    counts = [init.n]

    def make(state, gated, seq_part):
        n = init.n if state is None else state[4]
        return Trainer(init if state is None else None, cams, targets, rp, gate if gated else None,
                       max(4096, capacity_per_gaussian * n), gated=gated, sequence=seq_part,
                       state=state)

    tr = make(None, False, seq[:1])
    gs = torch.zeros(tr.n, device=tr.dev)
    cnt = torch.zeros(tr.n, dtype=torch.int32, device=tr.dev)
    d_view = torch.zeros(1, dtype=torch.int32, device=tr.dev)
    slot = torch.zeros(1, dtype=torch.int32, device=tr.dev)
    for t in range(densify_until):
        v = int(seq[t])
        d_view.fill_(v)
        tr.iteration(v, d_view, slot)
        sk.densify_stats([cams[v]], tr.n, rp, tr.ws, tr.cap, gs, cnt)
        if (t + 1) % densify_every == 0:
            planes, m, vv, n_new = densify_step(tr, dp, gs, cnt, rng)
            if log is not None:
                log(f"densify at {t + 1}: {tr.n} -> {n_new}")
            tr = make((planes, m, vv, tr.step_count, n_new, tr.deg), False, seq[:1])
            gs = torch.zeros(n_new, device=tr.dev)
            cnt = torch.zeros(n_new, dtype=torch.int32, device=tr.dev)
            counts.append(n_new)
    flags, _, _ = tr.status()
    post = make((tr.planes, tr.m, tr.v, tr.step_count, tr.n, tr.deg), True,
                seq[densify_until:densify_until + post_iters])
    for _ in range(post_iters):
        post.step()
    torch.cuda.synchronize()
    b, t_seen = post.backward_count()
    return {"counts": counts, "n": post.n, "status_densify": flags, "status_post": post.status()[0],
            "post_backward": b, "post_iterations": t_seen, "trainer": post}
