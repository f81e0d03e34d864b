"""Benchmark: Lanczos steps/s and H.v bandwidth on one MI355X.

A "step" is one Lanczos iteration (Alg. 1 loop body): the up-part kernel, the
down-part/diagonal/recurrence kernel with its partial dot products, the scalar
reduction and the vector update.  The default workload is the 4x4 periodic
Hubbard model at half filling (8 up + 8 down, dim 165,636,900, t=1, U=4) from a
seeded uniform(-1,1) start vector, float64 (the plain method); the mixed form
(float32 vectors, float64 scalars) is timed beside it.  The down species' basis
is taken in hop-count order (ed_hop_order; --basis-order ascending for the
paper's order) and the up species' in band order (ed_band_order; --up-order
ascending for the paper's): the same H up to a permutation of the vector
elements, with the start vector permuted alike, so the run has the same a_j,
b_j and E0.
Inputs are resident in HBM before the timed region; as in the paper's protocol
no transfer is timed.

Beside the step rate the line carries: the roofline of the dominant kernel
(HIP events inside this run), time-to-E0 at stated accuracy for plain float64,
mixed and learned starts at a held-out U (the network trained on the
method's own ground states at U = 1..8) with the ground state's observables,
the 64-instance batched launch against the same instances run one by one
(plain float64 and mixed) and 256 small instances batched against one by one,
the 18-site chain at 9 + 9 (2.36e9 states), the
one-species runs, the complex-amplitude checkerboard, the paper's own 18-site
workloads beside its K40 times, and the oracle timed on the host cores.

Prints ONE JSON line on stdout (progress lines go to stderr).  Options:
--steps K --warmup W (timed / untimed steps), --gpus N (only 1 is supported:
the method runs on one GPU), --no-cpu-baseline, --no-learned, --no-batch,
--no-scale, --no-single, --no-complex, --no-paper-shapes, --basis-order,
--up-order.
"""

import argparse
import json
import os
import sys
import time
from math import comb

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "Lanczos steps/s + H·v HBM GB/s, 4x4 Hubbard 8↑8↓, plain vs mixed/learned"
KERNELS = ("k_up", "k_down", "k_reduce", "k_update", "k_norm")


def hv_bytes(h, es):
    """Algorithmic HBM bytes of one H.v: x read once, y written once, plus each species' table and basis,
    B_hv = 2 p D + sum over species of D_sigma (W_sigma e + 8) with e the table entry size.  The up part T that
    the step's first kernel writes and its second reads back is an intermediate of this design, not an operand
    of H.v, so it is not counted."""
    D = h.dim
    tabs = sum(t.dim * (t.width * t.entry_bytes + 8) for t in (h.up, h.dn))
    return 2 * es * D + tabs


def kernel_bytes(h, es):
    """Bytes each step kernel moves by design (every operand once; the traffic it must move as written).

    k_up reads x and writes the up part: 2 p D plus the up table.
    k_down reads x, the up part and f_{j-1}, writes q: 4 p D plus the down table
    and both bases.  k_update reads q and f_j (and f_{j-1} in the mixed form)
    and writes f_{j+1}.  k_reduce and k_norm read a few hundred KB of partial sums."""
    D = h.dim
    tab_up = h.dim_up * h.up.width * h.up.entry_bytes
    tab_dn = h.dim_dn * h.dn.width * h.dn.entry_bytes
    states = 8 * (h.dim_up + h.dim_dn)
    upd = (4 if es == 4 else 3) * es * D
    return {"k_up": 2 * es * D + tab_up, "k_down": 4 * es * D + tab_dn + states,
            "k_reduce": 8 * 8 * h.dim_up, "k_update": upd, "k_norm": 8 * 8192}


def time_run(h, x, warmup, steps, n_kernel_samples):
    import torch
    total = warmup + steps + n_kernel_samples + 2
    run = h.lanczos(total)
    run.init(x)
    for _ in range(warmup):
        run.step()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        run.step()
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    import numpy as np
    per = np.zeros(5)
    for _ in range(n_kernel_samples):
        per += run.step_timed()
    per /= max(n_kernel_samples, 1)
    st = run.read()
    if st["steps"] != warmup + steps + n_kernel_samples or st["status"] not in (0,):
        raise RuntimeError("run did not complete every step: %r" % ({k: st[k] for k in ("steps", "status")},))
    return ms, dict(zip(KERNELS, per.tolist())), st


# Rows longer than this many states are gathered from global memory by the down part, not from LDS;
# there the ascending order's locality counts for more than the padding chunks the hop order drops
# (measured: the one-species 30-site torus ran 25% slower in FP64 in hop order).
LDS_ROW_STATES = 19456


def dn_order_for(args, dim_dn, cplx=False):
    """The down species' basis order for a run: --basis-order where FP64 rows sit in LDS, else ascending."""
    return args.basis_order if dim_dn * (2 if cplx else 1) <= LDS_ROW_STATES else "ascending"


def species_tables(ed, n_sites, bonds, n_up, n_dn, dev, dn_order, up_order="ascending", **kw):
    """(up, down) SpinTables: the up species in up_order, the down species in dn_order."""
    up = ed.SpinTables(n_sites, bonds, n_up, dev, order=up_order, **kw)
    if n_dn == n_up and dn_order == up_order:
        return up, up
    return up, ed.SpinTables(n_sites, bonds, n_dn, dev, order=dn_order, **kw)


def start_in_order(h, x_host, dev):
    """The seeded start vector (ascending order of both species) on the device, in h's basis order."""
    import torch
    x = torch.from_numpy(x_host).to(dev, h.torch_dtype)
    return h.to_basis_order(x) if h.order_bits else x


# the step kernels' sources: the traffic record is valid only for these exact bytes (of ed_device.hip, the part
# above the line that opens its host side: the step kernels and their launch shapes)
TRAFFIC_SOURCES = ("ed_device.hip", "ed_common.h", "ed_launch.h")
HOST_SIDE_MARK = b"// ---------------------------------------------------------------------------\n// Host side of the runs:"


def traffic_source_hash():
    """sha256 prefix of the step kernels' sources, as measured_traffic.json records it."""
    import hashlib
    here = os.path.join(ROOT, "paper_1511_00863_amd", "csrc")
    parts = []
    for f in TRAFFIC_SOURCES:
        b = open(os.path.join(here, f), "rb").read()
        if f == "ed_device.hip":
            cut = b.find(HOST_SIDE_MARK)
            if cut < 0:
                raise OSError("ed_device.hip has no host-side mark")
            b = b[:cut]
        parts.append(b)
    return hashlib.sha256(b"".join(parts)).hexdigest()[:16]


def measured_traffic(dtype, kernel, workload_name, basis_order, up_order="ascending"):
    """HBM bytes per launch from the committed counter record, if it matches this kernel source, workload and
    the two species' basis orders."""
    here = os.path.join(ROOT, "paper_1511_00863_amd")
    try:
        rec = json.load(open(os.path.join(here, "measured_traffic.json")))
        digest = traffic_source_hash()
    except OSError:
        return None
    if (digest != rec.get("source_sha256_prefix") or rec.get("workload") != workload_name
            or rec.get("basis_order_down", "ascending") != basis_order
            or rec.get("basis_order_up", "ascending") != up_order):
        return None
    return rec["kernels"].get(dtype, {}).get(kernel)


def scale_block(args):
    """Lanczos steps/s on the 18-site chain at 9 + 9 (D = 48620^2 = 2,363,904,400): a sector whose
    complex double-precision vector (38 GB) no coprocessor of the paper's day could hold, run here in
    float64 (18.9 GB per vector) and in the mixed form, with 32-bit tables (48620 states per species)."""
    import torch
    import paper_1511_00863_amd as ed
    from synth import workload
    wl = workload("ring18_9x9")
    dev = "cuda:0"
    # 48620-state rows, beyond LDS: the down species in band order, where the down part stages each
    # 8192-state column block with its neighbours in LDS (k_down_win over the species' row windows)
    tab, tdn = species_tables(ed, wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, dev, "band", args.up_order)
    out = {"workload": wl.name, "dim": tab.dim * tdn.dim, "U": wl.U, "table_entry_bytes": tab.entry_bytes,
           "basis_order": {"up": tab.order, "down": tdn.order},
           "start": "uniform(-1/2,1/2) from torch's device generator, seed %d, drawn in the run's order" % wl.seed}
    for dtype in ("f64", "f32"):
        h = ed.Hamiltonian(tab, tdn, wl.t, wl.U, dtype)
        src = ed.api.apply_tuned_tile(h, tune_if_missing=False)
        g = torch.Generator(device=dev)
        g.manual_seed(wl.seed)
        x = torch.rand(h.dim, dtype=h.torch_dtype, device=dev, generator=g).sub_(0.5)
        ms, per, _ = time_run(h, x, 2, args.scale_steps, 2)
        es = 8 if dtype == "f64" else 4
        out[dtype] = {"steps_per_s": 1000.0 / ms, "ms_per_step": ms, "kernel_ms": per,
                      "GB_per_vector": es * h.dim / 1e9, "tile": {"id": h.tile, "source": src, **h.tile_params()}}
        del x, h
        torch.cuda.empty_cache()
    del tab, tdn
    torch.cuda.empty_cache()
    return out


def single_block(args):
    """One spin species, the shape of the paper's one-species benchmarks: the 26-site chain with 13
    particles (D = 10,400,600) and a 30-site periodic lattice with 9 (D = 14,307,150).  All particles
    in the down species, so H x is the down-part kernel over one row of length D, split into column
    blocks, with no up part.  Algorithmic bytes of that kernel per launch: the start vector, f_{j-1}
    and q once each, the table's nonzeros (entries of H) and the states.  Read bytes: the same with the
    table chunks the kernel reads in place of the nonzeros: each wavefront's own chunk count
    (ed_wave_chunks) where the kernel takes it, else every chunk of the padded ELL rows."""
    import numpy as np
    import torch
    import paper_1511_00863_amd as ed
    from synth import start_vector, workload
    dev = "cuda:0"
    out = {}
    for name in ("ring26_0x13", "torus5x6_0x9"):
        wl = workload(name)
        up, dn = species_tables(ed, wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, dev, "ascending")   # one row of D
        x_host = start_vector(wl.seed, up.dim * dn.dim)
        rec = {"dim": up.dim * dn.dim, "table_stride": dn.stride, "table_entry_bytes": dn.entry_bytes,
               "basis_order": dn.order}
        for dtype in ("f64", "f32"):
            h = ed.Hamiltonian(up, dn, wl.t, wl.U, dtype)
            src = ed.api.apply_tuned_tile(h, tune_if_missing=False)
            x = start_in_order(h, x_host, dev)
            ms, per, _ = time_run(h, x, 3, args.single_steps, 3)
            es = 8 if dtype == "f64" else 4
            eb = dn.entry_bytes
            nonzeros = int(dn.table["nnz"].sum())
            # the chunk counts apply except in FP64 on 32-bit tables of more than 4 chunks
            wch = dn.dev_wch is not None and not (es == 8 and eb == 4 and dn.stride > 32)
            tab_read = (int(ed.wave_chunks(dn.table["nnz"]).astype(np.int64).sum()) * 64 * 8 * eb if wch
                        else h.dim * dn.stride * eb)
            vec_bytes = 3 * es * h.dim + 8 * h.dim
            t_dn = per["k_down"] * 1e-3
            rec[dtype] = {"steps_per_s": 1000.0 / ms, "ms_per_step": ms, "kernel_ms": per,
                          "k_down_alg_GBps": (vec_bytes + nonzeros * eb) / t_dn / 1e9,
                          "k_down_read_GBps": (vec_bytes + tab_read) / t_dn / 1e9,
                          "table_bytes_read": tab_read, "table_nonzero_bytes": nonzeros * eb,
                          "wave_chunk_counts": wch,
                          "tile": {"id": h.tile, "source": src, **h.tile_params()}}
            del x, h
            torch.cuda.empty_cache()
        out[name] = rec
        del up, dn, x_host
        torch.cuda.empty_cache()
    return out


def complex_block(args):
    """The paper's largest two-species checkerboard case: 18 sites, 5 + 5 (D = 73,410,624), complex
    nearest-neighbour amplitudes (synthetic values on the same lattice: 12 bonds per site), float64
    and the mixed form.  The paper's K40 took 712 ms (double) and 425 ms (single) per Lanczos
    iteration on this size (its checkerboard tables, 10 particles): context, other hardware."""
    import torch
    import paper_1511_00863_amd as ed
    from synth import start_vector_complex, workload
    wl = workload("checker18_5x5")
    dev = "cuda:0"
    tab, tdn = species_tables(ed, wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, dev, dn_order_for(args, comb(wl.n_sites, wl.n_dn), True),
                              amps=list(wl.amps))
    x_host = start_vector_complex(wl.seed, tab.dim * tdn.dim)
    out = {"workload": wl.name, "dim": tab.dim * tdn.dim, "U": wl.U, "table_stride": tab.stride,
           "n_amplitudes": tab.n_amps, "basis_order": {"up": "ascending", "down": tdn.order},
           "paper_k40_ms_per_step": {"f64": 712.0, "f32": 425.0}}
    for dtype in ("f64", "f32"):
        h = ed.Hamiltonian(tab, tdn, wl.t, wl.U, dtype)
        src = ed.api.apply_tuned_tile(h, tune_if_missing=False)
        x = start_in_order(h, x_host, dev)
        ms, per, _ = time_run(h, x, 3, args.complex_steps, 3)
        es = 16 if dtype == "f64" else 8
        dn_bytes = 4 * es * h.dim + tdn.dim * tdn.stride * 4 + 8 * 2 * tdn.dim
        out[dtype] = {"steps_per_s": 1000.0 / ms, "ms_per_step": ms, "kernel_ms": per,
                      "k_down_alg_GBps": dn_bytes / (per["k_down"] * 1e-3) / 1e9,
                      "up_alg_GBps": (2 * es * h.dim) / (per["k_up"] * 1e-3) / 1e9,
                      "tile": {"id": h.tile, "source": src, **h.tile_params()}}
        del x, h
        torch.cuda.empty_cache()
    return out


# The paper's per-iteration times on its K40 (ms; its tables for the 18-site lattices, N_up = N_dn = N/2)
PAPER_K40_MS = {
    "ring18": {2: (2.18, 2.26), 3: (2.70, 3.16), 4: (10.4, 17.7), 5: (88.4, 178.0)},        # (SP, DP)
    "checker18": {2: (2.20, 2.28), 3: (3.84, 5.17), 4: (40.8, 74.8), 5: (425.0, 712.0)},
}


def paper_shapes_block(args):
    """The paper's own two-species workloads: the 18-site chain (real hopping) and the 18-site checkerboard
    (complex amplitudes, synthetic values on the same lattice) at N_up = N_dn = 2..5, float64 and the
    mixed form, with the paper's K40 times beside them (context: other hardware; its FLOP model counts
    complex arithmetic for both lattices)."""
    import torch
    import paper_1511_00863_amd as ed
    from synth import ring_bonds, start_vector, start_vector_complex, workload
    dev = "cuda:0"
    cb = workload("checker18_5x5")
    out = {}
    for lat in ("ring18", "checker18"):
        for n in (2, 3, 4, 5):
            if lat == "ring18":
                tab, tdn = species_tables(ed, 18, ring_bonds(18), n, n, dev, dn_order_for(args, comb(18, n)))
                x_host = start_vector(11, tab.dim * tdn.dim)
            else:
                tab, tdn = species_tables(ed, 18, cb.bonds, n, n, dev, dn_order_for(args, comb(18, n), True),
                                          amps=list(cb.amps))
                x_host = start_vector_complex(11, tab.dim * tdn.dim)
            rec = {"dim": tab.dim * tdn.dim, "paper_k40_ms": {"f32": PAPER_K40_MS[lat][n][0],
                                                               "f64": PAPER_K40_MS[lat][n][1]}}
            for dtype in ("f64", "f32"):
                h = ed.Hamiltonian(tab, tdn, 1.0, 4.0, dtype)
                ed.api.apply_tuned_tile(h, tune_if_missing=False)
                x = start_in_order(h, x_host, dev)
                ms, _, _ = time_run(h, x, 2, args.paper_steps, 1)
                rec[dtype] = {"ms_per_step": ms, "vs_paper_k40": rec["paper_k40_ms"][dtype] / ms}
                del x, h
                torch.cuda.empty_cache()
            out["%s_%dx%d" % (lat, n, n)] = rec
            del tab, tdn, x_host
    return out


def observables_block(item, wl):
    """Occupation moments of a two-pass ground state (FP32 vector): wall time of ed_occupation_moments
    (two passes over the vector, synchronised) and the double occupancy and nearest-neighbour correlations."""
    import torch
    import paper_1511_00863_amd as ed
    ham, psi, _ = item
    ns = wl.n_sites
    g = ham.occupation_moments(psi, ns)          # warm-up
    best = None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = ham.occupation_moments(psi, ns)
        dt = (time.perf_counter() - t0) * 1e3
        best = dt if best is None else min(best, dt)
    c = ed.occupation_correlations(g, ns)
    a, b = wl.bonds[0]
    flip = ham.spin_flip_moments(psi, ns)         # one pass over psi per site; warm-up
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flip = ham.spin_flip_moments(psi, ns)
        times.append((time.perf_counter() - t0) * 1e3)
    flip_ms = float(np.median(times))
    ss = ed.spin_correlations(g, flip, ns)
    off = ~np.eye(ns, dtype=bool)
    return {"U": ham.U, "ms": best, "read_GBps": 2 * psi.numel() * psi.element_size() / (best * 1e6),
            "double_occupancy_per_site": float(c["docc"].mean()),
            "nn_bond": float(c["nn"][a, b]), "szsz_bond": float(c["szsz"][a, b]),
            "spin_flip_ms": flip_ms, "ss_bond": float(ss[a, b]), "ss_total": float(ss.sum()),
            "singlet_check_max_dev": float(np.max(np.abs(flip[off] - 2.0 * c["szsz"][off])))}


def time_to_e0_block(up, dn, wl, args):
    """Steps and wall ms to E0 at stated accuracy vs converged plain float64 Lanczos (the reference):
    plain float64 and mixed from the seeded random start, mixed and float64 from the learned start
    (network inference inside the timed region).  The network trains on ground states at U = 1..8."""
    import numpy as np
    import torch
    import paper_1511_00863_amd as ed
    from paper_1511_00863_amd import learned
    from synth import start_vector
    t0 = time.perf_counter()
    data = learned.training_data(up, dn, wl.t, [1, 2, 3, 4, 5, 6, 7, 8])
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net, losses, t_train = learned.train_network(data, iters=args.train_iters, batch=4096)
    obs = observables_block(data[3], wl)          # the U = 4 ground state
    del data
    torch.cuda.empty_cache()
    out = {"training": {"ground_states": 8, "data_s": t_data, "train_s": t_train, "iters": args.train_iters,
                        "batch": 4096, "loss_first": float(losses[:20].mean()), "loss_last": float(losses[-20:].mean())},
           "observables": obs, "held_out": []}
    t_cost = t_data + t_train
    saved = []
    for U in [float(u) for u in args.held_out.split(",")]:
        e_ref, ref_steps = learned.reference_energy(up, dn, wl.t, U, wl.seed)
        row = {"U": U, "e_ref": e_ref, "ref_steps": ref_steps}
        # overlap of each start with the ground state at this U (float64 two-pass vector)
        h = ed.Hamiltonian(up, dn, wl.t, U, "f64")
        ed.api.apply_tuned_tile(h, tune_if_missing=False)
        x = torch.from_numpy(start_vector(wl.seed, h.dim)).to("cuda:0", h.torch_dtype)
        _, _, psi = h.ground_state(x, min(800, ref_steps + 20))
        f_l = learned.learned_start(net, h, wl.seed)[0]
        row["overlap"] = {"random": abs(float(torch.dot(x, psi))) / float(torch.linalg.vector_norm(x)),
                          "learned": abs(float(torch.dot(f_l, psi))) / float(torch.linalg.vector_norm(f_l))}
        del h, x, psi, f_l
        torch.cuda.empty_cache()
        for dt, tol in (("f64", 1e-10), ("f32", 1e-6)):
            h = ed.Hamiltonian(up, dn, wl.t, U, dt)
            ed.api.apply_tuned_tile(h, tune_if_missing=False)
            x = torch.from_numpy(start_vector(wl.seed, h.dim)).to("cuda:0", h.torch_dtype)
            rnd = learned.time_to_e0(h, lambda: x.clone(), e_ref, tol)
            del x
            lrn = learned.time_to_e0(h, lambda: learned.learned_start(net, h, wl.seed)[0], e_ref, tol)
            name = "plain_f64" if dt == "f64" else "mixed"
            row[name + "_random"] = {"steps": rnd["steps"], "ms": rnd["ms"], "rel_tol": tol}
            row[name + "_learned"] = {"steps": lrn["steps"], "ms": lrn["ms"], "rel_tol": tol}
            if rnd["ms"] is not None and lrn["ms"] is not None:
                saved.append(rnd["ms"] - lrn["ms"])
            del h
            torch.cuda.empty_cache()
        out["held_out"].append(row)
    # the network's cost (training data from the method's own ground states, then training) against what
    # its start saves per solve, over the held-out runs above
    mean_saved = float(np.mean(saved)) if saved else None
    out["amortised"] = {"training_s": t_cost, "mean_saved_ms_per_solve": mean_saved,
                        "break_even_solves": (t_cost * 1e3 / mean_saved) if mean_saved and mean_saved > 0 else None}
    return out


def batch_block(args):
    """64 Hubbard instances on the 4x4 torus (U ~ U[0,8], N_up = N_dn in {3,4,5,6}) in one batched call
    (mixed form, |dE0| < 1e-6), against the same instances run one after another in plain float64 and in the
    mixed form.  The call puts the instances below 2^22 states in one persistent launch and runs the larger
    ones one by one after it (wall_ms); persistent_only_wall_ms is the call with every instance in the
    persistent launch."""
    import torch
    import paper_1511_00863_amd as ed
    from synth import batch_instances, start_vector, torus_bonds
    bonds = torus_bonds(4, 4)
    draws = batch_instances(64, 1000)
    tabs = {n: species_tables(ed, 16, bonds, n, n, "cuda:0", dn_order_for(args, comb(16, n)), args.up_order)
            for n in (3, 4, 5, 6)}
    hams = [ed.Hamiltonian(*tabs[n], 1.0, U, "f32") for (U, n, s) in draws]
    for h in hams:
        ed.api.apply_tuned_tile(h, tune_if_missing=False)
    f1s = [start_in_order(h, start_vector(s, h.dim), "cuda:0") for h, (U, n, s) in zip(hams, draws)]
    r = ed.ground_energy_batch(hams, f1s, 500, tol=1e-6)
    r = ed.ground_energy_batch(hams, f1s, 500, tol=1e-6)          # second call timed (warm)
    ed.ground_energy_batch(hams, f1s, 500, tol=1e-6, solo_dim=0)
    rp = ed.ground_energy_batch(hams, f1s, 500, tol=1e-6, solo_dim=0)
    n_solo = int(sum(h.dim >= ed.api.BATCH_SOLO_DIM for h in hams))
    del f1s
    torch.cuda.empty_cache()
    seq_ms, seq_e0 = 0.0, []
    for (U, n, s) in draws:
        h = ed.Hamiltonian(*tabs[n], 1.0, U, "f64")
        ed.api.apply_tuned_tile(h, tune_if_missing=False)
        x = start_in_order(h, start_vector(s, h.dim), "cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rr = h.ground_energy(x, 500, tol=1e-6, check_every=9)
        torch.cuda.synchronize()
        seq_ms += (time.perf_counter() - t0) * 1e3
        seq_e0.append(rr["e0"])
        del x
    seq_e0 = np.array(seq_e0)
    # the same instances one after another in the batch's own precision (mixed form), same tolerance
    mix_ms = 0.0
    for h, (U, n, s) in zip(hams, draws):
        x = start_in_order(h, start_vector(s, h.dim), "cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.ground_energy(x, 500, tol=1e-6, check_every=9)
        torch.cuda.synchronize()
        mix_ms += (time.perf_counter() - t0) * 1e3
        del x
    small = small_batch(tabs_for=lambda n: species_tables(ed, 16, bonds, n, n, "cuda:0", dn_order_for(args, comb(16, n)),
                                                          args.up_order))
    return {"basis_order": {"up": args.up_order, "down": args.basis_order}, "small_instances": small, "instances": 64, "total_dim": int(sum(h.dim for h in hams)), "wall_ms": r["wall_ms"],
            "graph_used": r["graph_used"], "converged": int((r["status"] == 0).sum()),
            "max_steps_used": int(r["steps"].max()), "sequential_plain_f64_ms": seq_ms,
            "sequential_mixed_ms": mix_ms,
            "max_rel_dev_vs_f64": float(np.max(np.abs(r["e0"] - seq_e0) / np.abs(seq_e0))),
            "solo_dim": ed.api.BATCH_SOLO_DIM, "instances_one_by_one": n_solo,
            "persistent_only_wall_ms": rp["wall_ms"], "persistent_only_converged": int((rp["status"] == 0).sum()),
            "persistent_only_max_rel_dev_vs_f64": float(np.max(np.abs(rp["e0"] - seq_e0) / np.abs(seq_e0)))}


def small_batch(tabs_for, n=256, seed=2000):
    """Many small instances, the batched launch's intended use: 256 Hubbard instances on the 4x4 torus with
    N_up = N_dn in {2, 3} (dims 14,400 and 313,600), U ~ U[0, 8], in one persistent launch against the same
    instances run one after another in the mixed form (same tolerance; tuned tiles where the cache has
    them, the default tile otherwise)."""
    import torch
    import paper_1511_00863_amd as ed
    from synth import batch_instances, start_vector
    draws = batch_instances(n, seed, fillings=(2, 3))
    tabs = {k: tabs_for(k) for k in (2, 3)}
    hams = [ed.Hamiltonian(*tabs[k], 1.0, U, "f32") for (U, k, s) in draws]
    for h in hams:
        ed.api.apply_tuned_tile(h, tune_if_missing=False)
    f1s = [start_in_order(h, start_vector(s, h.dim), "cuda:0") for h, (U, k, s) in zip(hams, draws)]
    ed.ground_energy_batch(hams, f1s, 500, tol=1e-6)
    r = ed.ground_energy_batch(hams, f1s, 500, tol=1e-6)
    seq_ms = 0.0
    for h, x in zip(hams, f1s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.ground_energy(x, 500, tol=1e-6, check_every=9)
        torch.cuda.synchronize()
        seq_ms += (time.perf_counter() - t0) * 1e3
    return {"instances": n, "fillings": [2, 3], "wall_ms": r["wall_ms"], "converged": int((r["status"] == 0).sum()),
            "sequential_mixed_ms": seq_ms, "speedup": seq_ms / r["wall_ms"]}


def cpu_baseline(wl, n_steps):
    """The oracle's float64 matrix-free Lanczos steps (NumPy/SciPy) on a sample of the workload."""
    import numpy as np
    from oracle.hamiltonian import Model
    from oracle.lanczos import lanczos
    from synth import start_vector
    host_cores = len(os.sched_getaffinity(0))
    blas_threads = os.environ.get("OMP_NUM_THREADS", "unset")
    m = Model(wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, wl.t, wl.U)
    _ = m.docc
    x = start_vector(wl.seed, m.dim)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):      # the BLAS dots too: the whole oracle on one thread
        t0 = time.perf_counter()
        lanczos(m.hv, x, n_steps)
        dt = time.perf_counter() - t0
    return {"value": n_steps / dt, "unit": "steps/s", "cores": 1, "kind": "oracle", "host_cores": host_cores,
            "sample": "%d float64 Lanczos steps of the oracle on the full %s workload (dim %d), %.1f s; "
                      "SciPy sparse-times-dense, NumPy elementwise and the BLAS dots (held to one thread) on one "
                      "thread of the host's %d (OMP_NUM_THREADS=%s outside it)"
                      % (n_steps, wl.name, m.dim, dt, host_cores, blas_threads)}


_T0 = None


def progress(what: str):
    """One progress line on stderr (stdout carries only the JSON line)."""
    global _T0
    if _T0 is None:
        _T0 = time.time()
    sys.stderr.write("[bench %6.1f s] %s\n" % (time.time() - _T0, what))
    sys.stderr.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="torus4x4_8x8")
    ap.add_argument("--kernel-samples", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in default tile instead of ed_tune")
    ap.add_argument("--no-learned", action="store_true", help="skip the time-to-E0 comparison with the learned start")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batched run")
    ap.add_argument("--train-iters", type=int, default=3000)
    ap.add_argument("--held-out", default="1.5,3.5,5.5,7.5", help="comma-separated held-out U values for time-to-E0")
    ap.add_argument("--no-scale", action="store_true", help="skip the 18-site 9+9 run (2.4e9 states)")
    ap.add_argument("--no-single", action="store_true", help="skip the one-species runs")
    ap.add_argument("--no-complex", action="store_true", help="skip the complex-amplitude checkerboard run")
    ap.add_argument("--no-paper-shapes", action="store_true", help="skip the paper's own 18-site workloads")
    ap.add_argument("--paper-steps", type=int, default=10)
    ap.add_argument("--complex-steps", type=int, default=20)
    ap.add_argument("--single-steps", type=int, default=20)
    ap.add_argument("--scale-steps", type=int, default=6)
    ap.add_argument("--basis-order", choices=("hops", "ascending"), default="hops",
                    help="basis order of the down species where its rows fit LDS")
    ap.add_argument("--up-order", choices=("band", "ascending"), default="band",
                    help="basis order of the up species in the timed step")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this method runs on one GPU; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1511_00863_amd as ed
    from synth import start_vector, workload

    wl = workload(args.workload)
    dev = "cuda:0"
    x64 = start_vector(wl.seed, 1)  # seed check (cheap); the full vector is drawn below
    del x64
    up = ed.SpinTables(wl.n_sites, wl.bonds, wl.n_up, dev)
    dn = up if wl.n_dn == wl.n_up else ed.SpinTables(wl.n_sites, wl.bonds, wl.n_dn, dev)
    # the timed step: down species in hop-count order, up species in band order (the same H up to a
    # permutation of the elements)
    order = dn_order_for(args, dn.dim)
    dn_run = dn if order == "ascending" else ed.SpinTables(wl.n_sites, wl.bonds, wl.n_dn, dev, order=order)
    up_run = up if args.up_order == "ascending" else ed.SpinTables(wl.n_sites, wl.bonds, wl.n_up, dev,
                                                                   order=args.up_order)
    x_host = start_vector(wl.seed, up.dim * dn.dim)

    results = {}
    for dtype in (("f64",) if args.no_mixed else ("f64", "f32")):
        h = ed.Hamiltonian(up_run, dn_run, wl.t, wl.U, dtype)
        x = h.to_basis_order(torch.from_numpy(x_host).to(dev, h.torch_dtype))   # the same start, reordered
        tile_src = "default"
        if not args.no_tune:           # the project's autotuner (cached per shape); outside the timed region
            tile_src = ed.api.apply_tuned_tile(h, x)
        ms, per, st = time_run(h, x, args.warmup, args.steps, args.kernel_samples)
        es = 8 if dtype == "f64" else 4
        kb = kernel_bytes(h, es)
        bhv = hv_bytes(h, es)
        progress("%s step timed: %.3f ms" % (dtype, ms))
        results[dtype] = {"ms_per_step": ms, "steps_per_s": 1000.0 / ms, "kernel_ms": per, "kernel_bytes": kb,
                          "hv_bytes": bhv, "step_floor_bytes": 3 * es * h.dim,
                          "tile": h.tile, "tile_params": h.tile_params(), "tile_src": tile_src,
                          "hv_alg_GBps": bhv / ((per["k_up"] + per["k_down"]) * 1e-3) / 1e9,
                          "step_floor_GBps": 3 * es * h.dim / (ms * 1e-3) / 1e9}
        del x, h
        torch.cuda.empty_cache()

    r64 = results["f64"]
    dom = max(KERNELS, key=lambda k: r64["kernel_ms"][k])
    # the dominant kernel against the algorithmic bytes of one H.v (2pD + tables)
    achieved = r64["hv_bytes"] / (r64["kernel_ms"][dom] * 1e-3) / 1e9
    t_hv = (r64["kernel_ms"]["k_up"] + r64["kernel_ms"]["k_down"]) * 1e-3
    traffic = {k: measured_traffic("f64", k, wl.name, dn_run.order, up_run.order) for k in ("k_up", "k_down")}
    hv_counter = (traffic["k_up"] + traffic["k_down"]) if None not in traffic.values() else None
    line = {
        "metric": METRIC,
        "value": r64["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "lattice": "4x4 periodic square" if wl.n_sites == 16 else wl.name,
                   "n_up": wl.n_up, "n_dn": wl.n_dn, "dim": up.dim * dn.dim, "t": wl.t, "U": wl.U,
                   "start": "uniform(-1,1), seed %d" % wl.seed,
                   "basis_order": {"up": up_run.order, "down": dn_run.order}},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic("f64", dom, wl.name, dn_run.order, up_run.order),
                     "bytes": "one H.v's algorithmic bytes, 2pD + tables = %d, over this kernel's mean time"
                              % r64["hv_bytes"]},
        "hv_pair": {"ms": t_hv * 1e3, "alg_GBps": r64["hv_bytes"] / t_hv / 1e9,
                    "frac": r64["hv_bytes"] / t_hv / 1e9 / HBM_PEAK_GBPS,
                    "counter_bytes": hv_counter,
                    "counter_frac": (hv_counter / t_hv / 1e9 / HBM_PEAK_GBPS) if hv_counter else None},
        "hv_alg_GBps": r64["hv_alg_GBps"],
        "step_floor_frac": r64["step_floor_GBps"] / HBM_PEAK_GBPS,
        "kernel_ms": r64["kernel_ms"],
        "tile": {"id": r64["tile"], "source": r64["tile_src"], **r64["tile_params"]},
    }
    if "f32" in results:
        r32 = results["f32"]
        line["mixed"] = {"dtype": "f32 vectors, f64 scalars", "steps_per_s": r32["steps_per_s"],
                         "ms_per_step": r32["ms_per_step"], "hv_alg_GBps": r32["hv_alg_GBps"],
                         "kernel_ms": r32["kernel_ms"], "step_floor_frac": r32["step_floor_GBps"] / HBM_PEAK_GBPS,
                         "tile": {"id": r32["tile"], "source": r32["tile_src"], **r32["tile_params"]}}
    if not args.no_learned:
        progress("time to E0 (training the start-vector network)")
        line["time_to_e0"] = time_to_e0_block(up, dn, wl, args)
    if not args.no_batch:
        progress("batch")
        line["batch"] = batch_block(args)
    if not args.no_scale:
        progress("18-site 9+9 scale run")
        line["scale"] = scale_block(args)
    if not args.no_single:
        progress("one-species runs")
        line["single_species"] = single_block(args)
    if not args.no_complex:
        progress("complex-amplitude checkerboard run")
        line["complex"] = complex_block(args)
    if not args.no_paper_shapes:
        progress("the paper's 18-site workloads")
        line["paper_shapes"] = paper_shapes_block(args)
    if not args.no_cpu_baseline:
        progress("CPU baseline (the oracle)")
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
