#!/usr/bin/env python3
"""Throughput of the PORTA hot path on one MI355X.

One step at the 256x256x128 precision instance (160 rays, 101 frequencies):
the FP32 short-characteristics BESSER sweep of every ray and frequency with
the fused FP64 J^K_Q / Lambda* integration, the FP64 statistical-equilibrium
update that rewrites the emissivities for the next iteration, and the FP32
reverse-sweep adjoint of an emergent-Stokes loss sum (I_top - target)^2
(gradients with respect to eta_I, the propagation matrix and the
emissivities).  The upward rays go range by range: a range is swept keeping
every plane and reversed at once, and the downward rays are swept after them;
where those planes do not fit in device memory, one forward sweep keeps every
C-th plane and the adjoint recomputes the rest.  Inputs are seeded synthetic
fields already resident in HBM.  Prints one JSON line on stdout.

After the timed steps (FP32 runs only, untimed): one FP32 and one FP64 sweep of the
same FP32-rounded inputs, whose largest differences over every emergent Stokes vector
and every point's J^K_Q go to `detail.precision`, then the FP64 sweep and step rates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12   # unpacked FP32 VALU, lane instructions/s
# kernels whose rocprofv3 VALU-busy figure shows them bound by the vector ALU rather than
# by HBM (the 9-point Bezier sweep, 78% busy at 3.2 TB/s); the others are reported
# against HBM
ALU_BOUND_KERNELS = ("k_sweep_plane<float, 1>",)
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--ray-batch", type=int, default=None,
                    help="rays swept together in the forward sweep and in the adjoint "
                         "(default 40; with --faces 0, every ray of a hemisphere)")
    ap.add_argument("--adjoint-ray-batch", type=int, default=0,
                    help="rays per batch in the adjoint (default: --ray-batch)")
    ap.add_argument("--checkpoint-stride", type=int, default=11,
                    help="checkpoint stride of the shared schedule")
    ap.add_argument("--schedule", default="auto", choices=["auto", "interleaved", "shared"],
                    help="interleaved: each range of upward rays is swept keeping every plane, "
                         "then reversed at once (no recompute); shared: one forward sweep keeps "
                         "every C-th plane and the adjoint recomputes the others; auto: "
                         "interleaved when its checkpoints fit in device memory")
    ap.add_argument("--range-rays", type=int, default=0,
                    help="upward rays per range of the interleaved schedule (0: the most, up "
                         "to 16, whose checkpoints fit)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--interp", default="bilinear", choices=["bilinear", "bezier2d"],
                    help="upwind/downwind interpolation (bezier2d: the 9-point monotonic "
                         "Bezier, forward and adjoint)")
    ap.add_argument("--stokes", type=int, default=4, choices=[4, 1],
                    help="4: Stokes-vector transfer; 1: the unpolarized (intensity-only) "
                         "problem (sweep only, with --no-adjoint)")
    ap.add_argument("--control", default="besser", choices=["besser", "parabolic"],
                    help="control point of the Bezier step: BESSER or the parabolic "
                         "(DELOPAR) rule (sweep only, with --no-adjoint)")
    ap.add_argument("--faces", action="store_true",
                    help="M and P on the first face of the grid each ray crosses, vertical "
                         "ones included (sweep only, with --no-adjoint)")
    ap.add_argument("--faces-chunk", type=int, default=0,
                    help="with --faces: frequencies per block of the first-face kernel "
                         "(0: as many as its LDS holds)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=-1,
                    help="row tiles per XCD per round (-1: the library default)")
    ap.add_argument("--no-fp64-rate", action="store_true",
                    help="skip the extra FP64 sweep used for the FP32-vs-FP64 rate")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32 sweep compared with the first FP64 sweep (profiles "
                         "use it, so that the FP32 kernels' launches are those of the step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB device-to-device first (counter calibration for profiles)")
    ap.add_argument("--cpu-pairs", type=int, default=48,
                    help="(ray, frequency) pairs of the workload swept by the CPU oracle")
    args = ap.parse_args()
    if args.ray_batch is None:
        # the first-face kernel's blocks are (ray, frequency chunk) pairs over a whole
        # plane: a hemisphere's rays in one launch fill the chip
        args.ray_batch = 0 if args.faces else 40
    return args


def sweep_launch_bytes(cfg, nrb, elem, nst=4):
    """Algorithmic HBM bytes of one plane launch of the sweep kernel: the upwind
    Stokes vector (nst components) read and the new one written per update, three
    planes of the 13 transfer coefficients, and the FP64 read-modify-write of the 10 J
    values of the previous plane."""
    np_ = cfg.nx * cfg.ny
    updates = nrb * cfg.nfreq * np_
    return updates * 2 * nst * elem + 3 * np_ * 13 * elem + np_ * 10 * 8 * 2, updates


def adjoint_launch_bytes(cfg, nrb, elem):
    """Algorithmic HBM bytes of one plane launch of the adjoint kernel: per update the
    adjoint of the plane above (or the seed) and the forward state of the plane below
    read and the new adjoint written; per node and ray the 33 partials written (in the
    sweep precision); three planes of the 13 transfer coefficients."""
    np_ = cfg.nx * cfg.ny
    updates = nrb * cfg.nfreq * np_
    return updates * 12 * elem + nrb * np_ * 33 * elem + 3 * np_ * 13 * elem, updates


KERNEL_SYMBOLS = {
    "k_sweep_plane<float, 0>": "_ZN5porta13k_sweep_planeIfLi0EEEvNS_9PlaneArgsIT_EE",
    "k_sweep_plane<double, 0>": "_ZN5porta13k_sweep_planeIdLi0EEEvNS_9PlaneArgsIT_EE",
    "k_adjoint_plane<float, 0>": "_ZN5porta15k_adjoint_planeIfLi0EEEvNS_7AdjArgsIT_EE",
    "k_adjoint_gather<float, 0>": "_ZN5porta16k_adjoint_gatherIfLi0EEEvNS_10GatherArgsIT_EE",
    "k_sweep_plane<float, 1>": "_ZN5porta13k_sweep_planeIfLi1EEEvNS_9PlaneArgsIT_EE",
    "k_sweep_plane_i<float>": "_ZN5porta15k_sweep_plane_iIfEEvNS_9PlaneArgsIT_EE",
    "k_sweep_plane_faces<float>": "_ZN5porta19k_sweep_plane_facesIfEEvNS_9FacesArgsIT_EE",
    "k_faces_setup<float>": "_ZN5porta13k_faces_setupIfEEvNS_9FacesArgsIT_EE",
    "k_adjoint_plane<float, 1>": "_ZN5porta15k_adjoint_planeIfLi1EEEvNS_7AdjArgsIT_EE",
    "k_adjoint_gather<float, 1>": "_ZN5porta16k_adjoint_gatherIfLi1EEEvNS_10GatherArgsIT_EE",
    "k_bez9_tgather<float>": "_ZN5porta14k_bez9_tgatherIfEEvNS_11TGatherArgsIT_EE",
}


def _amdgcn_code_objects(data):
    """The gfx950 ELF images inside the offload bundles of a host shared library."""
    import struct
    out, i, magic = [], 0, b"__CLANG_OFFLOAD_BUNDLE__"
    while (i := data.find(magic, i)) >= 0:
        n = struct.unpack_from("<Q", data, i + 24)[0]
        off = i + 32
        for _ in range(n):
            o, sz, tl = struct.unpack_from("<QQQ", data, off)
            triple = data[off + 24:off + 24 + tl]
            off += 24 + tl
            if b"amdgcn" in triple and sz:
                out.append(data[i + o:i + o + sz])
        i += len(magic)
    return out


def _elf_symbol_bytes(elf, name):
    """Bytes of a sized symbol of an ELF64 image (its machine code for a kernel)."""
    import struct
    shoff = struct.unpack_from("<Q", elf, 0x28)[0]
    shentsize, shnum = struct.unpack_from("<HH", elf, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + k * shentsize) for k in range(shnum)]
    want = name.encode()
    for sec in secs:
        if sec[1] != 2:                      # SHT_SYMTAB
            continue
        strtab = secs[sec[6]]
        for k in range(sec[5] // 24):
            st_name, _, _, shndx, value, size = struct.unpack_from("<IBBHQQ", elf, sec[4] + 24 * k)
            a = strtab[4] + st_name
            if size and elf[a:elf.index(b"\0", a)] == want:
                home = secs[shndx]
                fo = home[4] + (value - home[3])
                return elf[fo:fo + size]
    return None


def kernel_code_sha256(kernel, lib_path=None):
    """SHA-256 of a kernel's gfx950 machine code in the built library, or None."""
    import hashlib
    from paper_1307_4217_amd import porta
    sym = KERNEL_SYMBOLS.get(kernel)
    path = lib_path or porta.LIB_PATH
    if sym is None or not os.path.exists(path):
        return None
    for co in _amdgcn_code_objects(open(path, "rb").read()):
        b = _elf_symbol_bytes(co, sym)
        if b is not None:
            return hashlib.sha256(b).hexdigest()
    return None


def counter_workload(cfg, prec_name, schedule, nrb, range_rays):
    """The workload string under which the counters of a run are committed."""
    w = f"{cfg.nx}x{cfg.ny}x{cfg.nz} grid, {cfg.nrays} rays, {cfg.nfreq} frequencies, " \
        f"{'FP32' if prec_name == 'f32' else 'FP64'}"
    if schedule == "interleaved":
        return w + f", interleaved ranges of {range_rays} upward rays, downward ray batch {nrb}"
    return w + f", ray batch {nrb}"


def measured_counters(kernel, workload):
    """The committed counter record of a kernel for a workload (HBM bytes per launch from
    FETCH_SIZE / WRITE_SIZE, VALU busy), or None if there is none or the kernel's machine
    code differs from the one the counters were taken on."""
    import glob
    for path in sorted(glob.glob(os.path.join(PROFILES, "hbm_counters_*.json"))):
        rec = json.load(open(path))
        if rec.get("workload") != workload:
            continue
        k = rec["kernels"].get(kernel)
        if k is not None and k.get("code_sha256") == kernel_code_sha256(kernel):
            return k
    return None


def precision_report(it32, it64, j32, j64, nst):
    """Largest errors of an FP32 sweep against the FP64 sweep of the same FP32-rounded
    inputs: relative on I and absolute on Q/I, U/I, V/I over every top point, upward ray
    and frequency; J^K_Q (rows 0-8) relative to J^0_0 and Lambda-bar relative, at every
    point.  Compared ray by ray, in FP64, on the device."""
    ei = ep = 0.0
    for r in range(it64.shape[0]):
        a, b = it32[r].double(), it64[r]
        ia, ib = (a[..., 0], b[..., 0]) if nst == 4 else (a, b)
        ei = max(ei, ((ia - ib).abs() / ib.abs()).max().item())
        if nst == 4:
            ep = max(ep, (a[..., 1:] / ia[..., None] - b[..., 1:] / ib[..., None])
                     .abs().max().item())
    ej = ((j32[:9] - j64[:9]).abs() / j64[0].abs()).max().item()
    el = ((j32[9] - j64[9]).abs() / j64[9].abs()).max().item()
    return {"reference": "FP64 sweep of the same FP32-rounded inputs on the GPU",
            "i_rel_max": ei, "pol_abs_max": ep if nst == 4 else None,
            "jkq_rel_j00_max": ej, "lbar_rel_max": el,
            "outputs": int(it64.numel() // (4 if nst == 4 else 1))}


def host_cpus():
    """Threads the CPU baseline may use: the process's CPU share (OMP_NUM_THREADS where the
    job sets it, else the CPUs this process may run on), and a description of the host."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    share = int(os.environ.get("OMP_NUM_THREADS") or 0) or avail or 1
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(share, avail or share), {"nproc": os.cpu_count(), "affinity": avail,
                                        "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
                                        "cpu_model": model}


def cpu_baseline(cfg, atm, q, pairs):
    from oracle import oracle as orc
    import numpy as np
    share, host = host_cpus()
    nthreads = max(1, min(share, pairs))
    rays = np.linspace(0, cfg.nrays - 1, pairs).round().astype(np.int32)
    freqs = np.linspace(0, cfg.nfreq - 1, pairs).round().astype(np.int32)
    op = orc.OracleProblem(atm, q)
    t0 = time.perf_counter()
    done = 0
    # groups of `nthreads` rays at one frequency each, so every thread sweeps one pair
    for i in range(0, pairs, nthreads):
        rs = rays[i:i + nthreads]
        fs = freqs[i:i + 1]
        orc.fs_sweep(op, rays=rs, freqs=fs, want_j=True, want_itop=True, nthreads=nthreads)
        done += len(rs) * len(fs)
    dt = time.perf_counter() - t0
    per_pair = cfg.nx * cfg.ny * (cfg.nz - 1)     # node updates of one (ray, freq) pair
    upd = done * per_pair
    # and one thread on two of the pairs
    t1 = time.perf_counter()
    orc.fs_sweep(op, rays=rays[:2], freqs=freqs[:1], want_j=True, want_itop=True, nthreads=1)
    dt1 = time.perf_counter() - t1
    return {"value": upd / dt, "unit": "point*ray*freq updates/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{done} (ray, freq) pairs of the {cfg.nx}x{cfg.ny}x{cfg.nz} grid, FP64 "
                      f"sweep + J ({upd:.3e} updates in {dt:.1f} s) on the {nthreads} "
                      f"threads of this job's CPU share",
            "single_thread_value": 2 * per_pair / dt1,
            "single_thread_sample": f"2 of those pairs on one thread ({dt1:.1f} s)",
            "host": host}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "has no multi-GPU path (the sweep would shard by frequency across GPUs with one "
              "FP64 all-reduce of J per iteration).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1307_4217_amd import inputs, porta
    from paper_1307_4217_amd import schedule as schedule_mod

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    cfg = inputs.CONFIGS[args.config]
    prec = porta.F32 if args.prec == "f32" else porta.F64
    tdt = torch.float32 if prec == porta.F32 else torch.float64
    elem = 4 if prec == porta.F32 else 8
    log(f"config {cfg.name}: {inputs.describe(cfg)}, {cfg.updates:.4e} updates per sweep")
    atm = inputs.make_atmosphere(cfg, seed=0)
    q = inputs.make_quadrature(cfg)
    hg = porta.HostGrid.from_inputs(atm, q)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    kappa, prop, emis = t(atm.kappa, tdt), t(atm.propmat, tdt), t(atm.emis, tdt)
    s_a, s_b = t(atm.source, torch.float64), torch.empty((6, cfg.npoints), dtype=torch.float64,
                                                          device=dev)
    hanle = t(atm.hanle, torch.float64) if atm.hanle is not None else None
    bhat = t(atm.bhat, torch.float64) if atm.bhat is not None else None
    variant = args.stokes != 4 or args.control != "besser" or args.faces
    if variant and not args.no_adjoint:
        sys.exit("--stokes, --control and --faces time the sweep alone: add --no-adjoint")
    interp = porta.BEZIER2D if args.interp == "bezier2d" else porta.BILINEAR
    control = porta.CONTROL_PARABOLIC if args.control == "parabolic" else porta.CONTROL_BESSER
    nst = args.stokes
    opts = porta.options(ray_batch=args.ray_batch, block=args.block, xcd_remap=args.xcd_remap,
                         control=control, stokes=nst, faces=int(args.faces),
                         faces_chunk=args.faces_chunk)
    nrb = min(args.ray_batch, cfg.nmu * cfg.nchi) if args.ray_batch > 0 else cfg.nmu * cfg.nchi
    adj_opts = porta.options(ray_batch=args.adjoint_ray_batch or args.ray_batch, block=args.block,
                             xcd_remap=args.xcd_remap)
    ws_bytes = porta.workspace_size(hg, prec, porta.WS_SWEEP, 1, opts)
    nh = hg.nray_up
    schedule = "shared" if args.no_adjoint else args.schedule
    inter = None
    if schedule in ("auto", "interleaved"):
        # rays per range: checkpoints of every plane for them, plus the adjoint's
        # workspace beyond the sweep's, must fit beside what is already resident
        fixed = (2 * hg.nray_up * cfg.nfreq * cfg.npoints // cfg.nz * 4 * elem   # I_top, target
                 + 26 * cfg.npoints * (elem + 8) + ws_bytes)
        free = torch.cuda.mem_get_info()[0] - fixed - (8 << 30)
        range_rays = schedule_mod.fitting_range_rays(
            hg, prec, free, ws_bytes, limit=args.range_rays or 16, block=args.block,
            xcd_remap=args.xcd_remap)
        if range_rays:
            schedule = "interleaved"
        elif schedule == "interleaved":
            sys.exit("the interleaved schedule needs more device memory than is free")
        else:
            schedule = "shared"
    if schedule == "interleaved":
        # one workspace for every sweep and adjoint call, checkpoints for one range
        inter = schedule_mod.InterleavedSweep(hg, prec, range_rays, ray_batch=args.ray_batch,
                                              block=args.block, xcd_remap=args.xcd_remap,
                                              device=dev, interp=interp)
    elif not args.no_adjoint:
        # the sweep and the adjoint run one after the other and share one workspace
        ws_bytes = max(ws_bytes, porta.workspace_size(hg, prec, porta.WS_ADJOINT_CKPT,
                                                      args.checkpoint_stride, adj_opts))
    ws = inter.workspace if inter else torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ws_see = torch.empty(8 * ((cfg.npoints + 255) // 256) + 256, dtype=torch.uint8, device=dev)
    jkq = torch.empty((10, cfg.npoints), dtype=torch.float64, device=dev)
    itop = torch.empty((hg.nray_up, cfg.nfreq, cfg.ny, cfg.nx) + ((4,) if nst == 4 else ()),
                       dtype=tdt, device=dev)
    rc = torch.empty((), dtype=torch.float64, device=dev)
    log(f"workspace {ws.numel() / 1e9:.2f} GB, i_top {itop.numel() * elem / 1e9:.2f} GB")
    adj = not args.no_adjoint
    if adj:
        # loss target: emergent Stokes vectors of a seeded perturbed atmosphere
        tatm = inputs.perturbed_target_atmosphere(atm, seed=5)
        target = torch.empty_like(itop)
        tk, tp, te = t(tatm.kappa, tdt), t(tatm.propmat, tdt), t(tatm.emis, tdt)
        # swept with the launches of one step, so that a profile of the whole run holds
        # the step's mix of launch shapes
        for o in (inter.range_opts + [inter.down_opts] if inter else [opts]):
            porta.fs_sweep(hg, tk, tp, te, atm.i_bottom, atm.w2, prec=prec, interp=interp,
                           want_jkq=False, i_top=target, opts=o, workspace=ws)
        del tatm, tk, tp, te
        # 2 x target, so that the seed 2 (I_top - target) = lerp(I_top, 2 target, -1) is
        # one pass over I_top
        target2 = target.mul_(2.0)
        if inter:
            ckpt = inter.checkpoints
        else:
            # the forward sweep of each step keeps the upward rays' checkpoint planes for
            # the adjoint, which then only recomputes the planes between checkpoints
            ckpt = torch.empty(porta.checkpoint_size(hg, prec, args.checkpoint_stride) + 256,
                               dtype=torch.uint8, device=dev)
        ws_adj = ws
        g_k, g_p, g_e = torch.empty_like(kappa), torch.empty_like(prop), torch.empty_like(emis)
        log(f"{schedule} schedule: sweep/adjoint workspace {ws.numel() / 1e9:.2f} GB, "
            f"checkpoints {ckpt.numel() / 1e9:.2f} GB "
            + (f"(every plane of {inter.range_rays} rays at a time)" if inter
               else f"(stride {args.checkpoint_stride})"))

    ev = lambda: torch.cuda.Event(enable_timing=True)
    # the SEE writes the next emissivities into a second buffer, swapped in after the
    # adjoint so that the adjoint differentiates the sweep that produced I_top
    state = {"s_old": s_a, "s_new": s_b, "emis": emis, "emis_next": torch.empty_like(emis)}
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    class Mark:
        """HIP events around one library call, on torch's current stream."""

        def __init__(self, kind, marks):
            self.kind, self.marks = kind, marks

        def __enter__(self):
            self.a = ev()
            self.a.record()

        def __exit__(self, *exc):
            b = ev()
            b.record()
            self.marks.append((self.kind, self.a, b))

    def seed_rows(r, n, rows):
        # dL/dI_top of L = sum (I_top - target)^2 for these rows, in place
        rows.lerp_(target2[r:r + n], -1.0)

    def step_interleaved(times):
        emis_cur = state["emis"]
        marks = []
        g_k.zero_(), g_p.zero_(), g_e.zero_()
        inter.run(kappa, prop, emis_cur, atm.i_bottom, atm.w2, jkq, itop, seed_rows, g_k, g_p,
                  g_e, timer=lambda kind: Mark(kind, marks))
        with Mark("see", marks):
            porta.see_update(jkq, state["s_old"], atm.eps_c, atm.delta2, atm.w2, atm.planck,
                             hanle, bhat, kappa=kappa, emis_out=state["emis_next"], prec=prec,
                             s_new=state["s_new"], rc=rc, workspace=ws_see)
        state["s_old"], state["s_new"] = state["s_new"], state["s_old"]
        state["emis"], state["emis_next"] = state["emis_next"], state["emis"]
        times.append(marks)

    def step(times):
        if schedule == "interleaved":
            return step_interleaved(times)
        e = [ev() for _ in range(5)]
        emis_cur = state["emis"]
        e[0].record()
        porta.fs_sweep(hg, kappa, prop, emis_cur, atm.i_bottom, atm.w2, prec=prec,
                       interp=interp, jkq=jkq, i_top=itop, opts=opts, workspace=ws,
                       checkpoints=ckpt if adj else None,
                       checkpoint_stride=args.checkpoint_stride if adj else 0)
        e[1].record()
        porta.see_update(jkq, state["s_old"], atm.eps_c, atm.delta2, atm.w2, atm.planck, hanle,
                         bhat, kappa=kappa, emis_out=state["emis_next"], prec=prec,
                         s_new=state["s_new"], rc=rc, workspace=ws_see)
        e[2].record()
        if adj:
            # dL/dI_top of L = sum (I_top - target)^2, formed in place of I_top (not read
            # again this step), then the reverse sweep
            seed = itop.lerp_(target2, -1.0)
            e[3].record()
            g_k.zero_(), g_p.zero_(), g_e.zero_()
            porta.fs_adjoint(hg, kappa, prop, emis_cur, atm.i_bottom, seed, atm.w2, prec=prec,
                             interp=interp, checkpoint_stride=args.checkpoint_stride, g_kappa=g_k,
                             g_propmat=g_p, g_emis=g_e, opts=adj_opts, workspace=ws_adj,
                             checkpoints=ckpt)
        else:
            e[3].record()
        e[4].record()
        state["s_old"], state["s_new"] = state["s_new"], state["s_old"]
        state["emis"], state["emis_next"] = state["emis_next"], state["emis"]
        times.append([("sweep", e[0], e[1]), ("see", e[1], e[2]), ("seed", e[2], e[3]),
                      ("adjoint", e[3], e[4])])

    def split(marks):
        out = {"sweep": 0.0, "see": 0.0, "seed": 0.0, "adjoint": 0.0}
        for kind, a, b in marks:
            out[kind] += a.elapsed_time(b)
        return out

    for w in range(args.warmup):
        step([])
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(times)
        torch.cuda.synchronize()
        m = split(times[-1])
        log(f"step {k + 1}/{args.steps}: sweep {m['sweep']:.1f} ms, SEE {m['see']:.2f} ms, "
            f"adjoint {m['adjoint']:.1f} ms, R_c {rc.item():.3e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [split(e) for e in times]
    sweep_ms = sum(m["sweep"] for m in per) / args.steps
    see_ms = sum(m["see"] for m in per) / args.steps
    adj_ms = sum(m["adjoint"] for m in per) / args.steps
    step_ms = wall * 1e3 / args.steps
    # updates: one per node, ray and frequency on the nz - 1 planes after each ray's
    # boundary plane (the boundary plane is set, not solved)
    per_ray_freq = cfg.nx * cfg.ny * (cfg.nz - 1)
    fwd_updates = per_ray_freq * cfg.nrays * cfg.nfreq
    adj_updates = per_ray_freq * (cfg.nrays // 2) * cfg.nfreq if adj else 0
    value = (fwd_updates + adj_updates) * args.steps / wall

    # every plane launch of the sweep kernel in one step: its rays and algorithmic bytes
    if inter:
        shapes = inter.launch_ray_counts()
    else:
        shapes = [min(nrb, nh - r) for r in range(0, nh, nrb)] * 2
    launches = (cfg.nz - 1) * len(shapes)
    lbytes = (cfg.nz - 1) * sum(sweep_launch_bytes(cfg, n, elem, nst)[0]
                                for n in shapes) / launches
    lupd = fwd_updates / launches
    launch_ms = sweep_ms / launches
    achieved = lbytes / (launch_ms * 1e-3) / 1e9
    tname = "float" if elem == 4 else "double"
    kname = (f"k_sweep_plane_i<{tname}>" if nst == 1 else
             f"k_sweep_plane_faces<{tname}>" if args.faces else
             f"k_sweep_plane<{tname}, {1 if interp == porta.BEZIER2D else 0}>")
    workload = counter_workload(cfg, args.prec, schedule, nrb,
                                inter.range_rays if inter else 0)
    counters = (measured_counters(kname, workload) if args.block in (0, 256)
                and args.xcd_remap == -1 and args.faces_chunk == 0 else None)
    traffic = None if counters is None else counters["traffic_bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname,
                "valu_busy_pct": None if counters is None else counters.get("valu_busy_pct"),
                "launch_ms": round(launch_ms, 4), "bytes_per_launch": lbytes,
                "updates_per_launch": lupd}
    if kname in ALU_BOUND_KERNELS:
        # measured VALU-bound: the rate against the VALU issue peak, HBM beside it
        insts = None if counters is None else counters.get("sq_insts_valu_per_dispatch")
        lane = None if insts is None else insts * 64 / (launch_ms * 1e-3) / 1e12
        roofline.update({"bound": "alu", "achieved": None if lane is None else round(lane, 2),
                         "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instructions/s",
                         "frac": None if lane is None else round(lane / VALU_PEAK_TLANE, 4),
                         "hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}})
    if adj:
        # the adjoint kernel beside it: its launches carry the ray ranges (or adjoint
        # batches); the calls also hold the gathers of the partials, so this is a floor
        ashapes = ([n for _, n in inter.ranges] if inter else
                   [min(adj_opts.ray_batch or nh, nh - r)
                    for r in range(0, nh, adj_opts.ray_batch or nh)])
        alaunches = (cfg.nz - 1) * len(ashapes)
        abytes = (cfg.nz - 1) * sum(adjoint_launch_bytes(cfg, n, elem)[0]
                                    for n in ashapes) / alaunches
        alaunch_ms = adj_ms / alaunches
        aname = (f"k_adjoint_plane<{'float' if elem == 4 else 'double'}, "
                 f"{1 if interp == porta.BEZIER2D else 0}>")
        acounters = (measured_counters(aname, workload) if args.block in (0, 256)
                     and args.xcd_remap == -1 else None)
        # The adjoint kernel is bound by its vector ALU: its rate is the VALU instructions
        # of one launch (counted by rocprofv3 for this machine code) times 64 lanes over
        # the live launch time, against the unpacked FP32 issue peak of the part (one
        # lane instruction per lane per cycle: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz);
        # its HBM rate is reported beside it.
        insts = None if acounters is None else acounters.get("sq_insts_valu_per_dispatch")
        lane_rate = None if insts is None else insts * 64 / (alaunch_ms * 1e-3) / 1e12
        roofline_adjoint = {
            "bound": "alu", "kernel": aname,
            "achieved": None if lane_rate is None else round(lane_rate, 2),
            "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instructions/s",
            "frac": None if lane_rate is None else round(lane_rate / VALU_PEAK_TLANE, 4),
            "valu_busy_pct": None if acounters is None else acounters.get("valu_busy_pct"),
            "hbm": {"achieved": round(abytes / (alaunch_ms * 1e-3) / 1e9, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(abytes / (alaunch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "traffic": (None if acounters is None
                                else acounters["traffic_bytes_per_launch"])},
            "call_ms_per_launch": round(alaunch_ms, 4), "bytes_per_launch": abytes}
    extra = {"sweep_ms": round(sweep_ms, 2), "see_ms": round(see_ms, 3),
             "seed_ms": round(sum(m["seed"] for m in per) / args.steps, 2),
             "roofline_adjoint": roofline_adjoint if adj else None,
             "sweep_updates_per_s": fwd_updates / (sweep_ms * 1e-3),
             "effective_hbm_frac_34B": round(fwd_updates / (sweep_ms * 1e-3) * 34 / 8e12, 4),
             "adjoint_ms": round(adj_ms, 2),
             "adjoint_updates_per_s": (adj_updates / (adj_ms * 1e-3)) if adj else None,
             "adjoint_over_forward_time": round(adj_ms / sweep_ms, 3) if adj else None,
             "peak_device_memory_GB": round(torch.cuda.max_memory_allocated() / 1e9, 1)}
    if not args.no_fp64_rate and prec == porta.F32:
        del ws
        if adj:
            del ws_adj, ckpt
        inter = None   # holds the workspace and checkpoints of the interleaved schedule
        torch.cuda.empty_cache()
        # the FP32-rounded inputs, so that the first FP64 sweep is the reference of an
        # FP32 sweep of the same inputs (untimed)
        e32 = t(atm.emis, tdt)
        k64, p64, e64 = kappa.double(), prop.double(), e32.double()
        sshape = (hg.nray_up, cfg.nfreq, cfg.ny, cfg.nx) + ((4,) if nst == 4 else ())
        if not args.no_precision:
            ws32 = torch.empty(porta.workspace_size(hg, porta.F32, porta.WS_SWEEP, 1, opts),
                               dtype=torch.uint8, device=dev)
            it32 = torch.empty(sshape, dtype=torch.float32, device=dev)
            j32 = torch.empty_like(jkq)
            porta.fs_sweep(hg, kappa, prop, e32, atm.i_bottom, atm.w2, prec=porta.F32,
                           interp=interp, jkq=j32, i_top=it32, opts=opts, workspace=ws32)
            del ws32
        ws64 = torch.empty(porta.workspace_size(hg, porta.F64, porta.WS_SWEEP, 1, opts),
                           dtype=torch.uint8, device=dev)
        it64 = torch.empty(sshape, dtype=torch.float64, device=dev)
        porta.fs_sweep(hg, k64, p64, e64, atm.i_bottom, atm.w2, prec=porta.F64, interp=interp,
                       jkq=jkq, i_top=it64, opts=opts, workspace=ws64)
        if not args.no_precision:
            extra["precision"] = pr = precision_report(it32, it64, j32, jkq, nst)
            log(f"FP32 vs FP64 over {pr['outputs']:.3e} emergent Stokes vectors: I rel "
                f"{pr['i_rel_max']:.2e}, Q/I U/I V/I abs {pr['pol_abs_max'] or 0:.2e}; "
                f"J^K_Q {pr['jkq_rel_j00_max']:.2e} of J00, Lbar {pr['lbar_rel_max']:.2e}")
            del it32, j32
        del e32
        torch.cuda.empty_cache()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        porta.fs_sweep(hg, k64, p64, e64, atm.i_bottom, atm.w2, prec=porta.F64, interp=interp,
                       jkq=jkq, i_top=it64, opts=opts, workspace=ws64)
        b.record()
        torch.cuda.synchronize()
        ms64 = a.elapsed_time(b)
        extra["fp64_sweep_ms"] = round(ms64, 2)
        extra["fp64_sweep_updates_per_s"] = fwd_updates / (ms64 * 1e-3)
        extra["fp32_over_fp64_rate"] = round(ms64 / sweep_ms, 3)
        # the FP64 sweep kernel against HBM: its launches (ray batches of `nrb`), their
        # algorithmic bytes and, where committed, its counters
        shapes64 = [min(nrb, nh - r) for r in range(0, nh, nrb)] * 2
        n64 = (cfg.nz - 1) * len(shapes64)
        b64 = (cfg.nz - 1) * sum(sweep_launch_bytes(cfg, n, 8, nst)[0] for n in shapes64) / n64
        a64 = b64 / (ms64 / n64 * 1e-3) / 1e9
        k64name = ("k_sweep_plane_i<double>" if nst == 1 else
                   "k_sweep_plane_faces<double>" if args.faces else
                   f"k_sweep_plane<double, {1 if interp == porta.BEZIER2D else 0}>")
        c64 = (measured_counters(k64name, counter_workload(cfg, "f64", "shared", nrb, 0))
               if args.block in (0, 256) and args.xcd_remap == -1 and args.faces_chunk == 0
               else None)
        extra["fp64_roofline"] = {
            "bound": "hbm", "kernel": k64name, "achieved": round(a64, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(a64 / HBM_PEAK_GBS, 4),
            "traffic": None if c64 is None else c64["traffic_bytes_per_launch"],
            "valu_busy_pct": None if c64 is None else c64.get("valu_busy_pct"),
            "launch_ms": round(ms64 / n64, 4), "bytes_per_launch": b64}
        log(f"FP64 sweep {ms64:.1f} ms")
        if adj:
            # One FP64 step of the same schedule: the upward rays in ranges of 4 (every
            # plane of 4 rays in FP64 is 107 GB at 256x256x128), each swept keeping every
            # plane and reversed at once, the downward rays in batches, then the SEE
            del ws64
            torch.cuda.empty_cache()
            inter64 = schedule_mod.InterleavedSweep(hg, porta.F64, 4, ray_batch=args.ray_batch,
                                                    block=args.block,
                                                    xcd_remap=args.xcd_remap, device=dev,
                                                    interp=interp)
            target2_64 = target2.double()
            gk64, gp64, ge64 = (torch.zeros_like(k64), torch.zeros_like(p64),
                                torch.zeros_like(e64))
            e64_next = torch.empty_like(e64)
            s64_new = torch.empty_like(state["s_old"])
            marks64 = []

            def seed64(r, n, rows):
                rows.lerp_(target2_64[r:r + n], -1.0)

            torch.cuda.synchronize()
            t64 = time.perf_counter()
            inter64.run(k64, p64, e64, atm.i_bottom, atm.w2, jkq, it64, seed64, gk64, gp64,
                        ge64, timer=lambda kind: Mark(kind, marks64))
            with Mark("see", marks64):
                porta.see_update(jkq, state["s_old"], atm.eps_c, atm.delta2, atm.w2, atm.planck,
                                 hanle, bhat, kappa=k64, emis_out=e64_next, prec=porta.F64,
                                 s_new=s64_new, rc=rc, workspace=ws_see)
            torch.cuda.synchronize()
            wall64 = time.perf_counter() - t64
            m64 = split(marks64)
            extra["fp64_step_ms"] = round(wall64 * 1e3, 2)
            extra["fp64_step_updates_per_s"] = (fwd_updates + adj_updates) / wall64
            extra["fp64_step_sweep_ms"] = round(m64["sweep"], 2)
            extra["fp64_adjoint_ms"] = round(m64["adjoint"], 2)
            extra["fp64_adjoint_updates_per_s"] = adj_updates / (m64["adjoint"] * 1e-3)
            extra["fp32_over_fp64_step_rate"] = round(wall64 * 1e3 / step_ms, 3)
            extra["fp64_step"] = ("one step of the same schedule in FP64: upward rays in "
                                  "ranges of 4, stride-1 checkpoints, reversed at once; "
                                  "downward rays; SEE")
            log(f"FP64 step {wall64 * 1e3:.1f} ms (sweep {m64['sweep']:.1f}, adjoint "
                f"{m64['adjoint']:.1f}, SEE {m64['see']:.2f})")
            del inter64, target2_64
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample of the workload ...")
        cpu = cpu_baseline(cfg, atm, q, args.cpu_pairs)
        log(f"CPU oracle: {cpu['value']:.3e} updates/s on {cpu['cores']} threads")
    out = {
        "metric": "point*ray*freq updates/s (FP32 sweep + J + SEE, plus adjoint sweep)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == porta.F32 else "f64",
        "data": "synthetic (seeded two-level atmosphere with the paper's box geometry)",
        "config": {"workload": f"{cfg.nx}x{cfg.ny}x{cfg.nz} grid, {cfg.nrays} rays, "
                               f"{cfg.nfreq} freqs: Jacobi step (sweep+J+SEE)"
                               + (" + adjoint of the emergent-Stokes loss" if adj else "")
                               + "".join(f", {v}" for v, on in (
                                   ("9-point Bezier interpolation", interp == porta.BEZIER2D),
                                   ("unpolarized (intensity only)", nst == 1),
                                   ("parabolic control point", args.control == "parabolic"),
                                   ("M and P on the first face crossed", args.faces))
                                   if on),
                   "updates_per_step": fwd_updates + adj_updates,
                   "forward_updates": fwd_updates, "adjoint_updates": adj_updates,
                   "update_count": "one per node, ray and frequency on the nz-1 planes "
                                   "after each ray's boundary plane",
                   "ray_batch": nrb, "schedule": schedule,
                   "checkpoint_stride": 1 if schedule == "interleaved" else args.checkpoint_stride,
                   "adjoint_ray_batch": range_rays if schedule == "interleaved"
                   else adj_opts.ray_batch,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
