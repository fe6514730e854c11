"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2301_11828_amd.profiling trace DIR            # kernel-trace CSV -> per-kernel durations
    python -m paper_2301_11828_amd.profiling counters DIR_FETCH DIR_WRITE BYTES_COPY
                                                                  # FETCH_SIZE / WRITE_SIZE per dispatch
    python -m paper_2301_11828_amd.profiling pmc DIR              # mean of every counter per dispatch

DIR holds the CSV files rocprofv3 wrote with ``--output-format csv``.  The counter
summary calibrates FETCH_SIZE and WRITE_SIZE with the largest plain copy kernel
found in the same run (BYTES_COPY bytes read and written per dispatch) and reports
per-launch HBM traffic of each product kernel, together with a hash of the kernel
source so that stale numbers can be recognised.
"""
import collections
import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("passes.hip", "tile.hip", "epilogue.hpp", "fft_device.hpp", "passes.hpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    for k in ("k_tile_reg", "k_xfwd", "k_line_y", "k_line_z", "k_xinv", "k_yfwd", "k_yinv", "k_cg_sums", "k_group_sums",
              "k_dot_parts", "k_stretch", "k_scan", "k_emit", "k_tile"):
        if k in name:
            prec = "double" if "<double" in name else ("float" if "<float" in name else "")
            # chain passes: the BLOCK template flag false marks wave-owned teams
            wave = k in ("k_xfwd", "k_line_y", "k_line_z", "k_xinv", "k_yfwd", "k_yinv") and \
                "false" in name.split(k)[1][:40]
            return "%s<%s%s>" % (k, prec, ",wave" if wave else "")
    return name[:60]


def _key(r) -> str:
    """Kernel short name @ number of workgroups (tells launches of different plans apart)."""
    wg = 0
    for g, w in (("Grid_Size", "Workgroup_Size"), ("Grid_Size_X", "Workgroup_Size_X")):
        try:
            wg = int(r[g]) // max(1, int(r[w]))
            break
        except (KeyError, ValueError):
            continue
    return "%s@%d" % (_short(r["Kernel_Name"]), wg)


def trace(d: str):
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    durs = collections.defaultdict(list)
    for f in files:
        for r in csv.DictReader(open(f)):
            durs[_key(r)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    print("kernel@workgroups                            calls    avg_us    med_us    min_us")
    for k, v in sorted(durs.items(), key=lambda x: -sum(x[1])):
        v.sort()
        print("%-44s %5d %9.2f %9.2f %9.2f" % (k, len(v), sum(v) / len(v) / 1e3, v[len(v) // 2] / 1e3, v[0] / 1e3))
    print("source_hash: %s" % source_hash())


def _counter(d: str, name: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    vals = collections.defaultdict(list)
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == name:
                vals[(r["Kernel_Name"], _key(r))].append(float(r["Counter_Value"]))
    return vals


def counters(dfetch: str, dwrite: str, copy_bytes: float):
    fe, wr = _counter(dfetch, "FETCH_SIZE"), _counter(dwrite, "WRITE_SIZE")

    def copy_kernel(vals):
        cands = {k: v for k, v in vals.items() if "copybuffer" in k[0].lower()}
        return max(cands.items(), key=lambda kv: max(kv[1])) if cands else (None, None)

    ck, cf = copy_kernel(fe)
    _, cw = copy_kernel(wr)
    sf = (max(cf) * 1024.0 / copy_bytes) if cf else None
    sw = (max(cw) * 1024.0 / copy_bytes) if cw else None
    print("calibration copy kernel: %s, %.0f bytes read+written per dispatch" % (ck[0] if ck else None, copy_bytes))
    print("calibration: FETCH_SIZE reads %.4f x true bytes, WRITE_SIZE reads %.4f x" % (sf or float("nan"), sw or float("nan")))
    print("kernel@workgroups                            fetch_KiB  write_KiB  traffic_bytes_per_launch(calibrated)")
    rows = {}
    for k in sorted(set(fe) | set(wr), key=lambda kk: kk[1]):
        s = k[1]
        f = sum(fe.get(k, [0])) / max(len(fe.get(k, [1])), 1)
        w = sum(wr.get(k, [0])) / max(len(wr.get(k, [1])), 1)
        t = (f * 1024 / sf if sf else f * 1024) + (w * 1024 / sw if sw else w * 1024)
        rows[s] = t
        print("%-44s %10.1f %10.1f %14.0f" % (s, f, w, t))
    for k, t in rows.items():
        if k.startswith("k_"):
            print("traffic %s %.0f" % (k, t))
    print("source_hash: %s" % source_hash())
    return rows


def pmc(d: str):
    """Mean per dispatch of every collected counter, per product kernel."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for f in files:
        for r in csv.DictReader(open(f)):
            k = _key(r)
            if k.startswith("k_"):
                vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in vals.values() for c in v})
    print("kernel@workgroups".ljust(34) + "".join("%22s" % c for c in names))
    for k in sorted(vals):
        print(k.ljust(34) + "".join("%22.4g" % (sum(vals[k][c]) / len(vals[k][c]) if vals[k][c] else float("nan"))
                                    for c in names))
    print("source_hash: %s" % source_hash())


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], float(sys.argv[4]))
