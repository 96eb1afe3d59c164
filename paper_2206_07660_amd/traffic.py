"""HBM traffic of the dominant kernel from rocprofv3 counters.

Run the workload under two counter passes, then summarize:

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- \
        python3 -m paper_2206_07660_amd.traffic run
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT -o write -- \
        python3 -m paper_2206_07660_amd.traffic run
    python3 -m paper_2206_07660_amd.traffic summarize OUT profiles/traffic_counters.json

The workload is a plain device-to-device copy of a known size (calibration:
the counters read in KiB per dispatch; the factor that makes them equal to
the copy's 2 x N bytes is applied to every kernel) followed by one
polarization call (one q, Hermitian mode) and one self-energy call at the
si-4x4x4 shape, the launch configuration bench.py times, in fp64 and then in
the split-bf16 mode.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys

COPY_BYTES = 4 << 30
# kernel-name prefixes (tile shape and class tag of zgemm_k) of the launches bench.py times
CLASSES = {"pol_contract": "zgemm_k<2, 2, 1, 2, 2, 1,", "se_contract": "zgemm_k<2, 2, 1, 2, 3, 3,",
           "pol_producer": "zgemm_k<2, 2, 1, 2, 4, 2,", "se_producer": "zgemm_k<2, 2, 1, 2, 4, 4,",
           "se_final": "zgemm_k<1, 1, 4, 2, 2, 5,",
           # split-bf16 contractions of the GW_PREC_BF16X3 path
           "pol_contract_bf16x3": "bsgemm_k<2, 2, 2, 2, 1,", "se_contract_bf16x3": "bsgemm_k<2, 4, 4, 2, 3,"}


def run():
    import numpy as np
    import torch
    from . import gw
    from . import inputs as inp
    wl = inp.WORKLOADS["si-4x4x4"]
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    V = torch.zeros((wl.nk, wl.nk, wl.naux, wl.nao, wl.nao), dtype=torch.complex128, device="cuda")
    V[0].copy_(torch.from_numpy(inp.make_V_slab(wl, 0)))
    rng = np.random.default_rng(1)
    G = torch.from_numpy(inp.random_hermitian_tau(rng, wl.ntau, wl.nk, wl.nao, 0.1)).cuda()
    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, max_nq=1)
    gw.gw_set_hermitian(ctx, True)           # as in the scGW loop (G is Hermitian)
    P = torch.empty((1, wl.ntau, wl.naux, wl.naux), dtype=torch.complex128, device="cuda")
    gw.gw_polarization(ctx, V, G, 0, 1, P)
    S = torch.zeros((wl.ntau, wl.nk, wl.nao, wl.nao), dtype=torch.complex128, device="cuda")
    gw.gw_self_energy(ctx, V, G, P, 0, 1, S)
    torch.cuda.synchronize()
    ctx.close()
    # the same two calls in the split-bf16 mode (complex64 V)
    V32 = V.to(torch.complex64)
    del V
    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, max_nq=1, precision="bf16x3")
    gw.gw_set_hermitian(ctx, True)
    gw.gw_polarization(ctx, V32, G, 0, 1, P)
    gw.gw_self_energy(ctx, V32, G, P, 0, 1, S)
    torch.cuda.synchronize()
    ctx.close()
    print("traffic workload done", flush=True)


def _rows(outdir, tag):
    files = glob.glob(os.path.join(outdir, "**", f"{tag}*counter_collection.csv"), recursive=True)
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_kernel(rows, counter):
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        out.setdefault(name, []).append(float(r["Counter_Value"]))
    return out


def summarize(outdir, dest):
    from .build import source_hash          # the same hash bench.py checks
    fetch = _per_kernel(_rows(outdir, "fetch"), "FETCH_SIZE")
    write = _per_kernel(_rows(outdir, "write"), "WRITE_SIZE")

    def find(d, key):
        for name, vals in d.items():
            if key in name:
                return vals
        return None

    cf = find(fetch, "copyBuffer") or find(fetch, "elementwise") or find(fetch, "copy")
    cw = find(write, "copyBuffer") or find(write, "elementwise") or find(write, "copy")
    if not cf or not cw:
        raise SystemExit("copy kernel not found in the counter output")
    f_fetch = COPY_BYTES / (max(cf) * 1024.0)
    f_write = COPY_BYTES / (max(cw) * 1024.0)
    res = {"kernel_source_sha256": source_hash(), "copy_bytes": COPY_BYTES,
           "copy_fetch_kib": max(cf), "copy_write_kib": max(cw),
           "factor_fetch": f_fetch, "factor_write": f_write, "classes": {}}
    for cls, key in CLASSES.items():
        fv, wv = find(fetch, key), find(write, key)
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024.0 * f_fetch
        wb = sum(wv) / len(wv) * 1024.0 * f_write
        res["classes"][cls] = {"fetch_kib_per_launch": sum(fv) / len(fv),
                               "write_kib_per_launch": sum(wv) / len(wv),
                               "hbm_bytes_per_launch": fb + wb, "launches": len(fv)}
    with open(dest, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    if sys.argv[1] == "run":
        run()
    elif sys.argv[1] == "summarize":
        summarize(sys.argv[2], sys.argv[3])
