"""Summaries of rocprofv3 runs of bench.py, as short text and JSON for profiles/.

    python -m paper_0812_1282_amd.profiling trace DB --command CMD --out FILE.md
    python -m paper_0812_1282_amd.profiling traffic FETCH_DB WRITE_DB --copy-bytes N \
        --nodes N --command CMD --out FILE.json
    python -m paper_0812_1282_amd.profiling counters DB [DB ...] --command CMD --out FILE.md
    python -m paper_0812_1282_amd.profiling markers DB --command CMD --out FILE.md

`trace` tabulates a --kernel-trace database: calls, total, average and median
duration per kernel. `counters` tabulates the median per dispatch of every
counter in --pmc databases for the plain sweep launches of each format.
`markers` tabulates the library's roctx ranges from a --marker-trace database
(host time per entry point, graph capture and graph replay). `traffic` turns
two --pmc databases (FETCH_SIZE, then
WRITE_SIZE, in KiB per dispatch) into HBM bytes per sweep launch, each counter
scaled so that the device copy of a known size that the profiled command runs
first (bench.py --copy-calibration-mib) reads and writes exactly its size. The
JSON records a hash of the kernel sources, and bench.py reports the traffic
only while the sources still hash the same.

Reads only the SQLite output of rocprofv3 (tables `kernels`, `pmc_events`,
`regions`).
"""
import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
# The device code whose memory traffic the counters measure (the host side of
# the library only launches it).
SOURCES = ("csrc/lb_kernels.hip", "csrc/lb_internal.h")
STORAGE_NAMES = {0: "f64", 1: "f32", 2: "f16s", 3: "bf16s", 4: "f64c", 5: "f32c"}
# Bytes per lattice update that the stored layout moves when every stored word
# is read once and written once (the 16-bit formats keep f_0, f_1, f_3 and g_0
# in 32 bits: 44 B per node and buffer).
STORED_BYTES_PER_LU = {"f64": 288, "f32": 144, "f16s": 88, "bf16s": 88, "f64c": 208,
                       "f32c": 104, "f64ip": 288, "f32ip": 144}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


_SWEEP = re.compile(r"sweep_kernel<\s*(\d+)\s*,\s*(\d+)\s*,\s*(\d+)\s*,\s*(\w+)\s*,\s*(\w+)"
                    r"\s*(?:,\s*(\d+)\s*)?>")


def sweep_key(name):
    """(storage, collision, block_x, diag, tau_phi_one) of a sweep kernel name, else None.
    The in-place phases (read mode 1, 2) are named storage + "ip"."""
    m = _SWEEP.search(name)
    if not m:
        return None
    st = STORAGE_NAMES.get(int(m.group(1)), m.group(1))
    if m.group(6) and int(m.group(6)) > 0:
        st += "ip"
    return (st, int(m.group(2)), int(m.group(3)), m.group(4) == "true", m.group(5) == "true")


_BAND = re.compile(r"band_kernel<\s*(\d+)\s*,\s*(\d+)\s*,\s*(\w+)\s*>")


def band_key(name):
    """(in-place storage name, phase) of a band pre-pass kernel name, else None."""
    m = _BAND.search(name)
    if not m:
        return None
    return STORAGE_NAMES.get(int(m.group(1)), m.group(1)) + "ip", int(m.group(2)) - 1


def _phase(name):
    m = _SWEEP.search(name)
    return int(m.group(6)) - 1 if m and m.group(6) and int(m.group(6)) > 0 else None


def short_name(name):
    k = sweep_key(name)
    if k:
        st, coll, bx, diag, g1 = k
        ph = _phase(name)
        return (f"sweep {st} {'MRT' if coll else 'BGK'} block {bx}"
                f"{'' if ph is None else f' phase {ph}'}"
                f"{' +diag' if diag else ''}{' tau_phi=1' if g1 else ''}")
    b = band_key(name)
    if b:
        return f"band {b[0]} phase {b[1]}"
    return name.split("(")[0][:60]


def kernel_stats(db):
    c = sqlite3.connect(db).cursor()
    rows = c.execute("select name, duration from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, d in rows:
        agg[name].append(float(d))
    return agg


def trace_summary(db, command):
    agg = kernel_stats(db)
    lines = ["# rocprofv3 kernel trace", "", f"Command: `{command}`", "",
             "| kernel | calls | total ms | avg us | median us |", "|---|---|---|---|---|"]
    for name, ds in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        ds = sorted(ds)
        lines.append(f"| {short_name(name)} | {len(ds)} | {sum(ds) / 1e6:.3f} | "
                     f"{sum(ds) / len(ds) / 1e3:.2f} | {ds[len(ds) // 2] / 1e3:.2f} |")
    return "\n".join(lines) + "\n"


def per_dispatch(db, counter):
    c = sqlite3.connect(db).cursor()
    rows = c.execute("select name, counter_value from pmc_events where counter_name = ?",
                     (counter,)).fetchall()
    agg = collections.defaultdict(list)
    for name, val in rows:
        agg[name].append(float(val))
    return agg


def traffic_summary(fetch_db, write_db, copy_bytes, nodes, command):
    fetch = per_dispatch(fetch_db, "FETCH_SIZE")
    write = per_dispatch(write_db, "WRITE_SIZE")
    copy_f = [v for k, v in fetch.items() if COPY_KERNEL in k]
    copy_w = [v for k, v in write.items() if COPY_KERNEL in k]
    if not copy_f or not copy_w:
        raise SystemExit("no calibration copy kernel in the databases")
    f_fac = copy_bytes / (max(copy_f[0]) * 1024.0)
    w_fac = copy_bytes / (max(copy_w[0]) * 1024.0)
    out = {"command": command, "source_sha256": source_hash(), "nodes": nodes,
           "copy_bytes": copy_bytes, "fetch_factor": f_fac, "write_factor": w_fac,
           "formats": {}}
    # Per format, the kernels of one step: the plain sweep (no fused
    # diagnostics); in place, each phase's sweep and band pre-pass, averaged
    # over the two phases.
    groups = collections.defaultdict(list)
    for name, vals in fetch.items():
        k = sweep_key(name)
        if k and not k[3]:
            groups[k[0]].append(name)
        elif band_key(name):
            groups[band_key(name)[0]].append(name)

    def med(xs):
        xs = sorted(xs)
        return xs[len(xs) // 2]

    for st, names in groups.items():
        kern = {}
        for name in names:
            kern[short_name(name)] = {
                "dispatches": len(fetch[name]),
                "fetch_bytes": med(fetch[name]) * 1024.0 * f_fac,
                "write_bytes": med(write.get(name, [0.0])) * 1024.0 * w_fac}
        per_launch = 2.0 if st.endswith("ip") else 1.0   # two phases alternate
        fv = sum(k["fetch_bytes"] for k in kern.values()) / per_launch
        wv = sum(k["write_bytes"] for k in kern.values()) / per_launch
        stored = STORED_BYTES_PER_LU[st] * nodes
        out["formats"][st] = {"kernels": kern, "fetch_bytes": fv, "write_bytes": wv,
                              "stored_bytes": stored, "ratio": (fv + wv) / stored}
    return out


def counters_summary(dbs, command):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for db in dbs:
        c = sqlite3.connect(db).cursor()
        for name, cn, v in c.execute("select name, counter_name, counter_value from pmc_events"):
            k = sweep_key(name)
            if k and not k[3]:
                vals[k[0]][cn].append(float(v))
    names = sorted({cn for d in vals.values() for cn in d})
    lines = ["# rocprofv3 counters of the sweep (median per dispatch)", "",
             f"Command: `{command}`", "", "| counter | " + " | ".join(vals) + " |",
             "|---|" + "---|" * len(vals)]
    for cn in names:
        row = []
        for st in vals:
            xs = sorted(vals[st].get(cn, []))
            row.append(f"{xs[len(xs) // 2]:.4g}" if xs else "")
        lines.append(f"| {cn} | " + " | ".join(row) + " |")
    return "\n".join(lines) + "\n"


def marker_summary(db, command):
    """Calls, total, average and median host duration of each roctx range."""
    c = sqlite3.connect(db).cursor()
    agg = collections.defaultdict(list)
    for extdata, d in c.execute("select extdata, duration from regions"):
        try:
            name = json.loads(extdata).get("message", "?")
        except (TypeError, ValueError):
            name = str(extdata)
        agg[name].append(float(d))
    lines = ["# rocprofv3 marker trace (library roctx ranges, host time)", "",
             f"Command: `{command}`", "",
             "| range | calls | total ms | avg us | median us |", "|---|---|---|---|---|"]
    for name, ds in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        ds = sorted(ds)
        lines.append(f"| {name} | {len(ds)} | {sum(ds) / 1e6:.3f} | "
                     f"{sum(ds) / len(ds) / 1e3:.2f} | {ds[len(ds) // 2] / 1e3:.2f} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    q = sub.add_parser("traffic")
    q.add_argument("fetch_db")
    q.add_argument("write_db")
    q.add_argument("--copy-bytes", type=float, required=True)
    q.add_argument("--nodes", type=int, required=True)
    q.add_argument("--command", required=True)
    q.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    m = sub.add_parser("markers")
    m.add_argument("db")
    m.add_argument("--command", required=True)
    m.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        text = trace_summary(a.db, a.command)
    elif a.cmd == "markers":
        text = marker_summary(a.db, a.command)
    elif a.cmd == "counters":
        text = counters_summary(a.dbs, a.command)
    else:
        text = json.dumps(traffic_summary(a.fetch_db, a.write_db, a.copy_bytes, a.nodes,
                                          a.command), indent=1) + "\n"
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
