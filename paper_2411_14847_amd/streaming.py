"""Per-timestep streaming optimisation over the C ABI (Sec. 3.1-3.4).

A timestep starts from the previous timestep's Gaussians G = {G^base, G^var}.  With a dynamics
mask (the dynamic Gaussians' indices) it runs `iters` iterations of

    shift_apply(FWD) -> render_fwd (all views) -> L1 gradient + error maps -> render_bwd
    -> shift_apply(ADJOINT) -> adam_step over {dpos, drot} and every parameter of G^var,

where the offsets (dpos, drot) are either learnt directly for the dynamic Gaussians, or (shift =
"hash") produced by two hash-encoded deformation fields, H_dyn for the dynamic and H_st for the
static base Gaussians (Sec. 3.3), whose parameters Adam then updates instead;

bakes the shift into G, prunes G^var rows of very low opacity and appends Gaussians where the error
is large (densify_append).  The densified set G^var is kept between timesteps and erased every
`erase_every` timesteps (App. B); in the other timesteps an inheritance stage of `inherit_iters`
iterations first learns which of its Gaussians to keep (Sec. 3.2: a binary mask on opacity and
scale, straight-through gradient, mask loss) and removes the others.
The iteration can be captured once per timestep in a HIP graph and replayed (device-side Adam
step count; every buffer is preallocated, nothing in the loop allocates or synchronises).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import torch

from .api import Context, GaussianBuffers, RenderOut, zeroed_grads


@dataclass
class StreamConfig:
    iters: int = 100              # shift-stage steps per timestep (s2 = 100, Sec. 4.1)
    k_append: int = 5000          # Gaussians appended per timestep
    erase_every: int = 20         # G^var erased every 20 timesteps (App. B)
    gamma_err: float = 0.0        # error threshold of D_err (Sec. 3.4)
    tau_pos: float = 0.0          # historical-gradient thresholds of Eq. (4)
    tau_err: float = 0.0
    lr_dpos: float = 1e-3
    lr_drot: float = 1e-3
    lr_var: Dict[str, float] = field(default_factory=lambda: {
        "mean": 1e-3, "quat": 1e-3, "log_scale": 5e-3, "logit": 5e-2, "sh0": 2.5e-3, "sh_rest": 1.25e-4})
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    bg: tuple = (0.0, 0.0, 0.0)
    ssim_lambda: float = 0.0      # weight of the D-SSIM term of Eq. (3); 0 = L1 only
    use_graph: bool = False
    per_view: bool = False        # plain per-view loop (one render_fwd / render_bwd per camera)
    max_inflight: int = 0         # >0: at most this many iterations queued on the GPU at once, so
                                  # other streams sharing a hardware queue (serving) are not stuck
                                  # behind a whole timestep of replayed iterations
    seed: int = 0
    shift: str = "direct"         # "direct": per-Gaussian offsets of the dynamic group;
                                  # "hash": H_dyn / H_st deformation fields over every base Gaussian
    # (levels, features, log2 table rows, hidden units, N_min, N_max) of H_dyn and H_st; table
    # sizes of the N3DV setting (App. B)
    field_dyn: tuple = (16, 4, 16, 64, 16, 2048)
    field_st: tuple = (16, 2, 14, 64, 16, 2048)
    lr_field: float = 2e-3
    # selective inheritance (Sec. 3.2, App. B): s1 iterations (20 in the paper; 0 keeps every
    # G^var Gaussian), the mask-loss weight and the initial value of m (both not given by the
    # paper), Adam's learning rate for m
    inherit_iters: int = 0
    lambda_inher: float = 1e-6
    m_init: float = 0.5
    lr_mask: float = 0.05
    prune_min_opacity: float = 0.005  # G^var rows below this opacity are removed after each timestep


class Trainer:
    """Owns every device buffer of the loop; `g` is the live scene (capacity-sized planes)."""

    def __init__(self, ctx: Context, g: GaussianBuffers, cams, max_dynamic: int, cfg: StreamConfig):
        self.ctx, self.g, self.cams, self.cfg = ctx, g, list(cams), cfg
        dev = g.mean.device
        cap = g.capacity
        self.dev = dev
        # shifted scene: its own mean / quat planes, the other planes alias the live scene's
        self.gs = GaussianBuffers(torch.zeros_like(g.mean), torch.zeros_like(g.quat), g.log_scale, g.logit, g.sh,
                                  g.n, g.n_base, g.sh_degree)
        self.outs = [RenderOut.allocate(c, dev) for c in self.cams]
        self.dls = [torch.zeros(3, c.height, c.width, device=dev) for c in self.cams]
        self.errs = [torch.zeros(c.height, c.width, device=dev) for c in self.cams]
        self.ssim_scratch = ([torch.empty(9 * c.height * c.width, device=dev) for c in self.cams]
                             if cfg.ssim_lambda > 0.0 else None)
        self.targets = [torch.zeros(3, c.height, c.width, device=dev) for c in self.cams]
        # gradients and loss share one buffer, cleared by one fill per iteration; the historical
        # positional-gradient sums (Sec. 3.4) accumulate over the timestep's iterations
        self.zbuf, self.grads, (self.loss,) = zeroed_grads(g, [((1,), torch.float32)])
        self.gn = torch.zeros(cap, device=dev)
        self.cnt = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.n_app = torch.zeros(1, dtype=torch.int32, device=dev)
        self.d_step = torch.zeros(1, dtype=torch.int32, device=dev)
        md = max(1, max_dynamic)
        self.dyn_buf = torch.zeros(md, dtype=torch.int32, device=dev)
        self.dpos_buf = torch.zeros(3, md, device=dev)
        self.drot_buf = torch.zeros(4, md, device=dev)
        self.d_dpos_buf = torch.zeros(3, md, device=dev)
        self.d_drot_buf = torch.zeros(4, md, device=dev)
        self.mv_dyn = [torch.zeros(3, md, device=dev), torch.zeros(3, md, device=dev),
                       torch.zeros(4, md, device=dev), torch.zeros(4, md, device=dev)]
        self.m_var = g.zeros_like()
        self.v_var = g.zeros_like()
        self.nd = 0
        # selective inheritance: one value per row (G^var rows used), its gradient and moments,
        # and the opacity-logit / log-scale planes rendered under the mask
        self.m_inh = torch.zeros(cap, device=dev)
        self.dm_inh = torch.zeros(cap, device=dev)
        self.mv_inh = (torch.zeros(cap, device=dev), torch.zeros(cap, device=dev))
        self.lg_eff = torch.zeros(cap, device=dev)
        self.ls_eff = torch.zeros(3, cap, device=dev)
        self.n_kept = torch.zeros(1, dtype=torch.int32, device=dev)
        self.inherited = None
        self.fields = None
        if cfg.shift == "hash":
            self._init_fields()
        elif cfg.shift != "direct":
            raise ValueError(f"shift must be 'direct' or 'hash', not {cfg.shift!r}")
        self.graph = None
        self.graph_key = None
        self._inflight = []

    def _init_fields(self):
        """Two fields over the base Gaussians' bounding box (10% margin); reset to their initial
        (identity) parameters at every timestep.  Offsets are laid out [dynamic | static]."""
        from .api import HashField, geometric_res
        g, cfg, dev = self.g, self.cfg, self.dev
        nb = max(1, g.n_base)
        lo = g.mean[:, :nb].amin(dim=1).cpu()
        hi = g.mean[:, :nb].amax(dim=1).cpu()
        ext = (hi - lo).clamp_min(1e-3)
        lo, hi = (lo - 0.1 * ext).tolist(), (hi + 0.1 * ext).tolist()
        self.fields, self.field0, self.field_grads, self.field_mv = {}, {}, {}, {}
        for k, (L, F, lt, hid, nmin, nmax) in (("dyn", cfg.field_dyn), ("st", cfg.field_st)):
            f = HashField.init(geometric_res(nmin, nmax, L), F, lt, hid, lo, hi, dev, seed=cfg.seed + (k == "st"))
            self.fields[k] = f
            self.field0[k] = [t.clone() for t in f.arrays()]
            self.field_grads[k] = f.zeros_like()
            self.field_mv[k] = (f.zeros_like(), f.zeros_like())
        cap = g.capacity
        # H_dyn runs on a second stream with a context of its own (calls on one context may not
        # overlap): its few queries cannot fill the GPU alone, so they share it with H_st's
        self.ctx_dyn = Context(max_gaussians=cap, max_views=1, max_keys=1 << 10, max_tiles=16)
        self.side = torch.cuda.Stream()
        self.shift_buf = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.dpos_buf = torch.zeros(3, cap, device=dev)
        self.drot_buf = torch.zeros(4, cap, device=dev)
        self.d_dpos_buf = torch.zeros(3, cap, device=dev)
        self.d_drot_buf = torch.zeros(4, cap, device=dev)

    # ---- one iteration --------------------------------------------------------------------
    def _adam_groups(self):
        cfg, g = self.cfg, self.g
        nd = self.nd
        groups = []
        if self.fields is not None:
            for k, f in self.fields.items():
                m, v = self.field_mv[k]
                for p, gr, mm, vv in zip(f.arrays(), self.field_grads[k].arrays(), m.arrays(), v.arrays()):
                    groups.append((p, gr, mm, vv, cfg.lr_field))
        elif nd > 0:
            groups.append((self._dpos, self._d_dpos, self._m_dpos, self._v_dpos, cfg.lr_dpos))
            groups.append((self._drot, self._d_drot, self._m_drot, self._v_drot, cfg.lr_drot))
        lo, hi = g.n_base, g.n
        if hi > lo:
            lr = cfg.lr_var
            for name in ("mean", "quat", "log_scale"):
                P, Gr, M, V = (getattr(x, name) for x in (g, self.grads, self.m_var, self.v_var))
                for i in range(P.shape[0]):
                    groups.append((P[i, lo:hi], Gr[i, lo:hi], M[i, lo:hi], V[i, lo:hi], lr[name]))
            groups.append((g.logit[lo:hi], self.grads.logit[lo:hi], self.m_var.logit[lo:hi], self.v_var.logit[lo:hi],
                           lr["logit"]))
            for i in range(g.sh.shape[0]):
                groups.append((g.sh[i, lo:hi], self.grads.sh[i, lo:hi], self.m_var.sh[i, lo:hi],
                               self.v_var.sh[i, lo:hi], lr["sh0"] if i < 3 else lr["sh_rest"]))
        return groups

    # scenes from which H_dyn's queries run beside H_st's on the side stream by default
    OVERLAP_MIN_GAUSSIANS = 50_000

    def iteration(self, stream=None, overlap: Optional[bool] = None):
        """One shift-stage iteration on `stream`.  With `overlap`, H_dyn runs on a second stream
        beside H_st; without it, on `stream` too.  Once HIP has more than four hardware queues the
        fork and join cost about 1 ms per iteration, eager or replayed from a graph (1.3 ms per
        replayed 20-view iteration at 8 queues): the overlap pays for that only when the fields
        have many queries, so by default (None) it is used from OVERLAP_MIN_GAUSSIANS base
        Gaussians on (the 200k-Gaussian scene: 604 ms per timestep eager with it, 615 replayed
        without; the 7k-Gaussian rig: 180 ms eager with it, 62 replayed without), and graph
        capture passes False."""
        if overlap is None:
            overlap = self.g.n_base >= self.OVERLAP_MIN_GAUSSIANS
        ctx, g, gs, cfg = self.ctx, self.g, self.gs, self.cfg
        gs.n, gs.n_base = g.n, g.n_base
        cur = stream if stream is not None else torch.cuda.current_stream()
        if self.fields is not None:
            dyn_stream = self.side if overlap else cur
            nd, ns, F = self.nd, self.ns, self.fields
            for k in ("dyn", "st"):
                for t in self.field_grads[k].arrays():
                    t.zero_()
            if overlap:
                self.side.wait_stream(cur)
            self.ctx_dyn.hash_field_fwd(F["dyn"], g.mean, g.n_base, self._dyn, nd, self._dpos, self._drot, col=0,
                                        stream=dyn_stream)
            ctx.hash_field_fwd(F["st"], g.mean, g.n_base, self._st, ns, self._dpos, self._drot, col=nd, stream=stream)
            if overlap:
                cur.wait_stream(self.side)
        ctx.shift_fwd(g, gs, self._shift_idx, self._dpos, self._drot, stream=stream)
        self.zbuf.zero_()
        self._d_dpos.zero_()
        self._d_drot.zero_()
        if not cfg.per_view:
            if cfg.ssim_lambda > 0.0:
                ctx.render_fwd(gs, self.cams, cfg.bg, out=self.outs, stream=stream)
                ctx.fidelity_loss_grad(self.cams, [o.rgb for o in self.outs], self.targets, cfg.ssim_lambda, self.dls,
                                       self.errs, self.loss, scratch=self.ssim_scratch, stream=stream)
            else:
                ctx.render_fwd_l1(gs, self.cams, cfg.bg, self.targets, self.dls, self.errs, self.loss,
                                  out=self.outs, stream=stream)
            ctx.render_bwd(gs, self.cams, cfg.bg, self.outs, self.dls, self.grads, self.gn, self.cnt, stream=stream)
        else:
            V = len(self.cams)
            for v in range(V):
                sl = slice(v, v + 1)
                ctx.render_fwd(gs, self.cams[sl], cfg.bg, out=self.outs[sl], stream=stream)
                if cfg.ssim_lambda > 0.0:
                    ctx.fidelity_loss_grad(self.cams[sl], [self.outs[v].rgb], self.targets[sl], cfg.ssim_lambda,
                                           self.dls[sl], self.errs[sl], self.loss, scratch=self.ssim_scratch[sl],
                                           stream=stream)
                else:
                    ctx.l1_loss_grad(self.cams[sl], [self.outs[v].rgb], self.targets[sl], self.dls[sl], self.errs[sl],
                                     self.loss, stream=stream)
                with torch.cuda.stream(stream or torch.cuda.current_stream()):
                    self.dls[v].mul_(1.0 / V)
                ctx.render_bwd(gs, self.cams[sl], cfg.bg, self.outs[sl], self.dls[sl], self.grads, self.gn, self.cnt,
                               stream=stream)
        if int(self._shift_idx.numel()) > 0:
            ctx.shift_adjoint(g, self._shift_idx, self._drot, self.grads, self._d_dpos, self._d_drot, stream=stream)
        if self.fields is not None:
            dyn_stream = self.side if overlap else cur
            nd, ns, F = self.nd, self.ns, self.fields
            if overlap:
                self.side.wait_stream(cur)
            self.ctx_dyn.hash_field_bwd(F["dyn"], g.mean, g.n_base, self._dyn, nd, self._d_dpos, self._d_drot,
                                        self.field_grads["dyn"], col=0, stream=dyn_stream)
            ctx.hash_field_bwd(F["st"], g.mean, g.n_base, self._st, ns, self._d_dpos, self._d_drot,
                               self.field_grads["st"], col=nd, stream=stream)
            if overlap:
                cur.wait_stream(self.side)
        groups = self._adam_groups()
        if groups:
            ctx.adam_step(groups, cfg.beta1, cfg.beta2, cfg.eps, stream=stream, d_step=self.d_step)

    def autotune_tile(self, reps: int = 3, batches=(128, 64)) -> dict:
        """Picks the context's tile size and blend batch with the native autotuner on the current
        timestep's render (call after at least one iteration of the timestep, so the upstream
        gradients are real).  The graph of the timestep is re-captured at the next replay."""
        scratch = self.g.zeros_like()
        res = self.ctx.autotune_tile(self.gs, self.cams, self.cfg.bg, self.outs, self.dls, scratch, reps=reps,
                                     batches=batches)
        self.graph = None
        return res

    # ---- one timestep -----------------------------------------------------------------------
    def inheritance_stage(self):
        """Selective inheritance of G^var: cfg.inherit_iters iterations of mask -> render -> fidelity
        loss -> render_bwd -> straight-through adjoint -> Adam on m, then the masked rows are
        removed.  Returns (G^var rows before, rows kept)."""
        ctx, g, cfg = self.ctx, self.g, self.cfg
        nb, nv = g.n_base, g.n - g.n_base
        m = self.m_inh[:nv]
        dm = self.dm_inh[:nv]
        mm, vm = self.mv_inh[0][:nv], self.mv_inh[1][:nv]
        m.fill_(cfg.m_init)
        mm.zero_()
        vm.zero_()
        ge = GaussianBuffers(g.mean, g.quat, self.ls_eff, self.lg_eff, g.sh, g.n, g.n_base, g.sh_degree)
        for it in range(cfg.inherit_iters):
            self.zbuf.zero_()
            dm.zero_()
            ctx.inherit_apply(g, m, self.lg_eff, self.ls_eff)
            if cfg.ssim_lambda > 0.0:
                ctx.render_fwd(ge, self.cams, cfg.bg, out=self.outs)
                ctx.fidelity_loss_grad(self.cams, [o.rgb for o in self.outs], self.targets, cfg.ssim_lambda, self.dls,
                                       self.errs, self.loss, scratch=self.ssim_scratch)
            else:
                ctx.render_fwd_l1(ge, self.cams, cfg.bg, self.targets, self.dls, self.errs, self.loss, out=self.outs)
            ctx.render_bwd(ge, self.cams, cfg.bg, self.outs, self.dls, self.grads)
            ctx.inherit_adjoint(g, m, self.grads.logit, self.grads.log_scale, cfg.lambda_inher, dm, self.loss)
            ctx.adam_step([(m, dm, mm, vm, cfg.lr_mask)], cfg.beta1, cfg.beta2, cfg.eps, step=it + 1)
        ctx.compact_var(g, m, 0.0, self.n_kept)
        kept = int(self.n_kept.item())
        g.n = nb + kept
        return nv, kept

    def begin_timestep(self, t: int, dyn_idx: torch.Tensor):
        cfg, g = self.cfg, self.g
        self.inherited = None
        if t % cfg.erase_every == 0:
            g.n = g.n_base  # erase G^var
        elif cfg.inherit_iters > 0 and g.n > g.n_base:
            self.inherited = self.inheritance_stage()
        nd = int(dyn_idx.numel())
        self.nd = nd
        self.gn.zero_()
        self.cnt.zero_()
        for t_ in (*self.m_var.planes(), *self.v_var.planes()):
            t_.zero_()
        self.d_step.zero_()
        if self.fields is not None:
            return self._begin_fields(dyn_idx)
        self.dyn_buf[:nd] = dyn_idx
        for t_ in self.mv_dyn:
            t_.zero_()
        # contiguous views of the preallocated buffers used by the kernels for this timestep
        flat = lambda buf, rows: buf.view(-1)[:rows * nd].view(rows, nd)
        self._dyn = self.dyn_buf[:nd]
        self._shift_idx = self._dyn
        self._dpos, self._drot = flat(self.dpos_buf, 3), flat(self.drot_buf, 4)
        self._dpos.zero_()
        self._drot.zero_()
        self._drot[0] = 1.0
        self._d_dpos, self._d_drot = flat(self.d_dpos_buf, 3), flat(self.d_drot_buf, 4)
        self._m_dpos, self._v_dpos = flat(self.mv_dyn[0], 3), flat(self.mv_dyn[1], 3)
        self._m_drot, self._v_drot = flat(self.mv_dyn[2], 4), flat(self.mv_dyn[3], 4)

    def _begin_fields(self, dyn_idx: torch.Tensor):
        """Shift rows [dynamic | static] of the base set; fields back to their initial parameters."""
        g, nd = self.g, self.nd
        nb = g.n_base
        static = torch.ones(nb, dtype=torch.bool, device=self.dev)
        static[dyn_idx.long()] = False
        st = static.nonzero().view(-1).to(torch.int32)
        self.ns = int(st.numel())
        if self.ns + nd != nb:
            raise ValueError("dynamic indices must be distinct rows of the base set")
        self.shift_buf[:nd] = dyn_idx
        self.shift_buf[nd:nb] = st
        self._shift_idx = self.shift_buf[:nb]
        self._dyn, self._st = self.shift_buf[:nd], self.shift_buf[nd:nb]
        flat = lambda buf, rows: buf.view(-1)[:rows * nb].view(rows, nb)
        self._dpos, self._drot = flat(self.dpos_buf, 3), flat(self.drot_buf, 4)
        self._d_dpos, self._d_drot = flat(self.d_dpos_buf, 3), flat(self.d_drot_buf, 4)
        for k, f in self.fields.items():
            for dst, src in zip(f.arrays(), self.field0[k]):
                dst.copy_(src)
            for t_ in (*self.field_mv[k][0].arrays(), *self.field_mv[k][1].arrays()):
                t_.zero_()

    def set_targets(self, images: List[torch.Tensor]):
        for dst, src in zip(self.targets, images):
            dst.copy_(src)

    def _throttle(self):
        if self.cfg.max_inflight > 0:
            ev = torch.cuda.Event()
            ev.record()
            self._inflight.append(ev)
            if len(self._inflight) > self.cfg.max_inflight:
                self._inflight.pop(0).synchronize()

    def run_iterations(self, k: int):
        if not self.cfg.use_graph:
            for _ in range(k):
                self.iteration()
                self._throttle()
            return
        key = (self.g.n, self.nd)
        if self.graph is None or self.graph_key != key:
            # warm up on a side stream, then capture one iteration
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            step0 = self.d_step.clone()
            with torch.cuda.stream(s):
                self.iteration(stream=s, overlap=False)
            torch.cuda.current_stream().wait_stream(s)
            self.graph = torch.cuda.CUDAGraph()
            # thread-local capture: a serving thread may keep using the device meanwhile
            with torch.cuda.graph(self.graph, capture_error_mode="thread_local"):
                self.iteration(stream=torch.cuda.current_stream(), overlap=False)
            self.graph_key = key
            k -= 1  # the warm-up ran one real iteration; capture itself does not execute
            del step0
        for _ in range(k):
            self.graph.replay()
            self._throttle()

    def shift_final(self):
        """Shifted means and quaternions of the final parameters: the last iteration shifted G before
        its Adam step, so the shift is taken again from the updated offsets (or fields, whose
        offsets are recomputed) and the updated G^var rows."""
        g, gs = self.g, self.gs
        gs.n, gs.n_base = g.n, g.n_base
        if self.fields is not None:
            F = self.fields
            self.ctx_dyn.hash_field_fwd(F["dyn"], g.mean, g.n_base, self._dyn, self.nd, self._dpos, self._drot, col=0)
            self.ctx.hash_field_fwd(F["st"], g.mean, g.n_base, self._st, self.ns, self._dpos, self._drot, col=self.nd)
        self.ctx.shift_fwd(g, gs, self._shift_idx, self._dpos, self._drot)

    def end_timestep(self, t: int) -> int:
        """Bakes the shift into G and appends Gaussians; returns the number appended."""
        cfg, g, gs = self.cfg, self.g, self.gs
        n = g.n
        self.shift_final()
        g.mean[:, :n].copy_(gs.mean[:, :n])
        g.quat[:, :n].copy_(gs.quat[:, :n])
        self.pruned = 0
        if cfg.prune_min_opacity > 0.0 and g.n > g.n_base:
            self.ctx.compact_var(g, None, cfg.prune_min_opacity, self.n_kept)
            kept = int(self.n_kept.item())
            self.pruned = g.n - g.n_base - kept
            g.n = g.n_base + kept
        self.ctx.densify_append(g, self.errs, self.cams, self.gn, self.cnt, cfg.gamma_err, cfg.tau_pos, cfg.tau_err,
                                cfg.k_append, cfg.seed * 1_000_003 + t, self.n_app)
        k = int(self.n_app.item())
        # device-side errors of the timestep (a tile-key overflow truncates the lists of every
        # iteration after it): raised here, where the host has waited for the work anyway
        self.ctx.sync()
        if self.fields is not None:
            self.ctx_dyn.sync()
        g.n += k
        self.graph = None
        self._inflight.clear()  # the item() above waited for everything queued so far
        return k

    def timestep(self, t: int, dyn_idx: torch.Tensor, targets: List[torch.Tensor]) -> dict:
        t0 = time.perf_counter()
        self.set_targets(targets)
        self.begin_timestep(t, dyn_idx)
        first = None
        scale = 1.0 / len(self.cams) if self.cfg.per_view else 1.0  # per-view calls each add a view's mean
        if self.cfg.iters > 0:
            self.iteration()
            first = float(self.loss.item()) * scale
            self.run_iterations(self.cfg.iters - 1)
        last = float(self.loss.item()) * scale
        appended = self.end_timestep(t)
        torch.cuda.current_stream().synchronize()
        return {"t": t, "ms": (time.perf_counter() - t0) * 1e3, "loss_first": first, "loss_last": last,
                "appended": appended, "n": self.g.n, "inherited": self.inherited, "pruned": self.pruned}
