"""HBM traffic per kernel launch from rocprofv3 counter runs.

Two `rocprofv3 --pmc` passes over the same command (FETCH_SIZE, then WRITE_SIZE; both in KiB
per dispatch) and the same two passes over a plain device copy of known size give, per
kernel, the average bytes fetched from and written to HBM per launch, each scaled by the
factor that makes the copy's counters equal its known bytes.

    python -m paper_2310_19855_amd.pmc --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --copy-bytes N --command "..." --out profiles/traffic_field1080_plain.json
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_src_hash(key):
    """hash of the source that defines kernel k_<key>, the shared headers and the host sources
    (which lay out what the kernels read, e.g. the BVH); None for a kernel that is not the
    library's.  A traffic figure is only valid for the code it was taken on."""
    csrc = os.path.join(HERE, "csrc")
    files = sorted(os.listdir(csrc))
    owner = None
    for f in files:
        if f.endswith(".hip") and re.search(r"\bk_%s\b" % re.escape(key), open(os.path.join(csrc, f)).read()):
            owner = f
            break
    if owner is None:
        return None
    h = hashlib.sha256()
    for f in [owner] + [f for f in files if f.endswith(".hpp") or f.endswith(".cpp")]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_key(name):
    """short name of a library kernel (k_trace_probes<16>(...) -> trace_probes); other kernels
    keep their name up to the argument list"""
    m = re.search(r"\bk_(\w+?)\s*[<(]", name)
    if m:
        return m.group(1)
    return name.split("(")[0].strip()


def read_counter(run_dir, counter):
    """{kernel key: [value per dispatch]} for one counter from a rocprofv3 counter CSV"""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    out = {}
    for path in files:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                out.setdefault(kernel_key(row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
    return out


def build(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, command):
    f = read_counter(fetch_dir, "FETCH_SIZE")
    w = read_counter(write_dir, "WRITE_SIZE")
    cf = read_counter(copy_fetch_dir, "FETCH_SIZE")
    cw = read_counter(copy_write_dir, "WRITE_SIZE")
    # the copy kernel is the one launch set whose counters are largest
    ck = max(cf, key=lambda k: sum(cf[k]))
    copy_fetch_kib = sum(cf[ck]) / len(cf[ck])
    copy_write_kib = sum(cw[ck]) / len(cw[ck])
    sf = copy_bytes / (copy_fetch_kib * 1024.0)
    sw = copy_bytes / (copy_write_kib * 1024.0)
    kernels = {}
    for k in sorted(set(f) & set(w)):
        fb = sum(f[k]) / len(f[k]) * 1024.0 * sf
        wb = sum(w[k]) / len(w[k]) * 1024.0 * sw
        kernels[k] = {"dispatches": len(f[k]), "fetch_bytes": round(fb), "write_bytes": round(wb),
                      "bytes_per_launch": round(fb + wb), "src_hash": kernel_src_hash(k)}
    return {"command": command,
            "calibration": {"kernel": ck, "copy_bytes": copy_bytes, "fetch_kib": copy_fetch_kib,
                            "write_kib": copy_write_kib, "fetch_scale": sf, "write_scale": sw},
            "kernels": kernels}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    d = build(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.command)
    with open(a.out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d["calibration"]))
    for k, v in d["kernels"].items():
        print(f"{k:>16}: {v['bytes_per_launch'] / 1e6:10.2f} MB/launch over {v['dispatches']} dispatches")


if __name__ == "__main__":
    main()
