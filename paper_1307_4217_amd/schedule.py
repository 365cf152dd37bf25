"""Interleaved forward and reverse sweeps for a loss that sums over the upward rays.

When the loss is a sum over upward rays of functions of each ray's emergent Stokes
vectors (a least-squares misfit of I_top, for instance), the seed dL/dI_top of a ray
depends on that ray's rows of I_top alone.  The upward rays can then go range by
range: a range is swept keeping the state of every plane (checkpoint stride 1), its
seed is formed from its rows of I_top, and it is reversed at once from those planes,
so the adjoint recomputes nothing.  The downward rays, which the loss does not see,
are swept last; J adds up over all the calls.  Each range's checkpoints reuse one
buffer, whose size sets the number of rays per range.

Every step runs in the library (porta_fs_sweep, porta_fs_adjoint over ray ranges);
this module only orders the calls and owns the buffers.
"""
from __future__ import annotations

from contextlib import nullcontext

from . import porta


def fitting_range_rays(hg, prec, free_bytes, base_ws_bytes, limit=16, ray_batch=0, block=0,
                       xcd_remap=-1):
    """The largest number of upward rays per range (at most `limit`) whose stride-1
    checkpoints, plus the adjoint workspace beyond `base_ws_bytes`, fit in
    `free_bytes`; 0 if not even one ray does."""
    for n in range(min(limit, hg.nray_up), 0, -1):
        o = porta.options(ray_batch=n, block=block, xcd_remap=xcd_remap, ray_count=n)
        need = (porta.checkpoint_size(hg, prec, 1, o)
                + max(0, porta.workspace_size(hg, prec, porta.WS_ADJOINT_CKPT, 1, o)
                      - base_ws_bytes))
        if need <= free_bytes:
            return n
    return 0


class InterleavedSweep:
    """One formal solution of every ray with J, and the adjoint of a loss summed over
    the upward rays, for fixed grid, quadrature and precision.

    range_rays : upward rays per range (each range is one sweep call and one adjoint
                 call, every plane of its rays kept in between)
    ray_batch  : rays per launch for the downward rays (0: all of them)
    The buffers (checkpoints for one range and one workspace shared by all the calls)
    are allocated on construction.
    """

    def __init__(self, hg, prec, range_rays, ray_batch=40, block=0, xcd_remap=-1,
                 device="cuda", interp=porta.BILINEAR):
        import torch
        if range_rays < 1:
            raise ValueError("range_rays must be >= 1")
        self.hg, self.prec, self.interp = hg, prec, interp
        nh = hg.nray_up
        self.range_rays = min(range_rays, nh)
        self.ranges = [(r, min(self.range_rays, nh - r)) for r in range(0, nh, self.range_rays)]
        self.range_opts = [porta.options(ray_batch=self.range_rays, block=block,
                                         xcd_remap=xcd_remap, ray_first=r, ray_count=n)
                           for r, n in self.ranges]
        self.down_opts = porta.options(ray_batch=ray_batch, block=block, xcd_remap=xcd_remap,
                                       ray_first=nh, ray_count=nh)
        ws = max(porta.workspace_size(hg, prec, porta.WS_SWEEP, 1, self.down_opts),
                 porta.workspace_size(hg, prec, porta.WS_SWEEP, 1, self.range_opts[0]),
                 porta.workspace_size(hg, prec, porta.WS_ADJOINT_CKPT, 1, self.range_opts[0]))
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        self.checkpoints = torch.empty(
            max(porta.checkpoint_size(hg, prec, 1, self.range_opts[0]), 256), dtype=torch.uint8,
            device=device)

    @property
    def buffer_bytes(self):
        return self.workspace.numel() + self.checkpoints.numel()

    def launch_ray_counts(self):
        """Rays per launch of the sweep kernel over one run: each range once, then the
        downward batches."""
        nh = self.hg.nray_up
        rb = self.down_opts.ray_batch or nh
        return [n for _, n in self.ranges] + [min(rb, nh - r) for r in range(0, nh, rb)]

    def run(self, kappa, propmat, emis, i_bottom, w2, jkq, i_top, seed, g_kappa, g_propmat,
            g_emis, stream=None, timer=None):
        """Sweep every ray (J into `jkq`, overwritten; I_top of the upward rays into
        `i_top`) and add the loss gradients to g_kappa, g_propmat, g_emis.

        seed(r0, n, rows) is called after the sweep of upward rays [r0, r0 + n) with
        rows = i_top[r0:r0 + n]; it writes dL/dI_top of those rays into `rows` in place
        (I_top is not read again).  `timer(kind)`, if given, returns a context manager
        around each call, kind being "sweep", "seed" or "adjoint"."""
        t = timer or (lambda kind: nullcontext())
        hg, prec = self.hg, self.prec
        for i, (r, n) in enumerate(self.ranges):
            o = self.range_opts[i]
            with t("sweep"):
                porta.fs_sweep(hg, kappa, propmat, emis, i_bottom, w2, prec=prec,
                               interp=self.interp, jkq=jkq, accumulate=i > 0, i_top=i_top,
                               opts=o, workspace=self.workspace,
                               stream=stream, checkpoints=self.checkpoints, checkpoint_stride=1)
            with t("seed"):
                seed(r, n, i_top[r:r + n])
            with t("adjoint"):
                porta.fs_adjoint(hg, kappa, propmat, emis, i_bottom, i_top, w2, prec=prec,
                                 interp=self.interp, checkpoint_stride=1, g_kappa=g_kappa, g_propmat=g_propmat,
                                 g_emis=g_emis, opts=o, workspace=self.workspace,
                                 stream=stream, checkpoints=self.checkpoints)
        with t("sweep"):
            porta.fs_sweep(hg, kappa, propmat, emis, i_bottom, w2, prec=prec,
                           interp=self.interp, jkq=jkq, accumulate=True, want_itop=False,
                           opts=self.down_opts,
                           workspace=self.workspace, stream=stream)
