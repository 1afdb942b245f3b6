"""HBM traffic per kernel launch from rocprofv3 counter runs.

    python -m paper_1902_02508_amd.counters --fetch DIR --write DIR \\
        --copy-fetch DIR --copy-write DIR --copy-mib 512 --workload NAME --out FILE.md

Each DIR is the output directory of one ``rocprofv3 --pmc <counter>
--output-format csv -d DIR -o run`` run: FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) of the benchmark, and of ``bench.py --copy-calibration MIB``,
whose device-to-device copies move a known number of bytes. Each counter is
scaled by (known copy bytes) / (what it reads for the copy), so the figures
are bytes to and from HBM in the copy kernel's units. The summary records
the SHA-256 of the sources each kernel is built from; bench.py reports the
traffic only while those sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# kernel symbol fragment (name, or name with template arguments) ->
# (short name, sources it is compiled from)
_DF = ["k_dfilt.hip", "eles_internal.h"]
_FT = ["k_sder.hip", "eles_internal.h"]
KERNELS = {
    "k_xz": ("k_xz", ["k_xz.hip", "eles_internal.h"]),
    "k_xzm": ("k_xzm", ["k_xzm.hip", "eles_internal.h"]),
    "k_xzw": ("k_xzw", ["k_xzw.hip", "eles_internal.h"]),
    "k_ys": ("k_ys", ["k_ys.hip", "eles_internal.h"]),
    # the direct y pass of the stress, by arithmetic (FP32 / BF16 / BF16x3)
    "k_y<true, 0>": ("k_y_fp32", ["k_y.hip", "eles_internal.h"]),
    "k_y<true, 1>": ("k_y_bf16", ["k_y.hip", "eles_internal.h"]),
    "k_y<true, 2>": ("k_y_bf16x3", ["k_y.hip", "eles_internal.h"]),
    # differential filter: transforms (x with the products, z), y solves, epilogue
    "k_dfwd_lds<false, true>": ("dfilter_xf", _DF),
    "k_dfwd_lds<true, false>": ("dfilter_zf", _DF),
    "k_dsolve<true>": ("dfilter_y", _DF),
    "k_dinv_lds<true>": ("dfilter_zi", _DF),
    "k_dinv_lds<false>": ("dfilter_xi", _DF),
    "k_depi": ("dfilter_epi", _DF),
    # ... the same passes by fast transforms (keys ending in a comma match
    # every instance with these leading template arguments)
    "k_rfft<false, false,": ("dfilter_xf", _FT),
    "k_rfft<false, true,": ("dfilter_zf", _FT),
    "k_rfft<true, true,": ("dfilter_zi", _FT),
    "k_rfft<true, false,": ("dfilter_xi", _FT),
}
_SOURCES = {}
for _name, _srcs in KERNELS.values():
    _SOURCES.setdefault(_name, []).append(_srcs)


def source_hash(names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(CSRC, n), "rb") as fh:
            h.update(n.encode())
            h.update(fh.read())
    return h.hexdigest()


def _per_dispatch(directory: str, counter: str) -> dict:
    """{kernel short name or symbol: [KiB per dispatch, ...]}."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    out: dict = {}
    for fn in files:
        with open(fn, newline="") as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                # filed under the bare name and, for templates, also with
                # the template arguments
                m = re.search(r"(k_[a-z_0-9]+)(<[^>]*>)?", r["Kernel_Name"])
                keys = [m.group(1)] + ([m.group(1) + m.group(2)] if m.group(2) else []) if m else [r["Kernel_Name"]]
                for key in keys:
                    out.setdefault(key, []).append(float(r["Counter_Value"]))
    return out


def copy_scale(directory: str, counter: str, mib: int) -> float:
    """Known bytes / counter bytes for the plain copy dispatches."""
    d = _per_dispatch(directory, counter)
    vals = [v for k, vs in d.items() if "copy" in k.lower() for v in vs if v > 0]
    big = [v for v in vals if v * 1024 > 0.25 * mib * (1 << 20)]   # the calibration copies, not setup ones
    if not big:
        raise ValueError(f"no copy dispatch found in {directory}")
    measured = sum(big) / len(big) * 1024.0
    return mib * (1 << 20) / measured


def summarize(fetch, write, copy_fetch, copy_write, mib):
    sf = copy_scale(copy_fetch, "FETCH_SIZE", mib)
    sw = copy_scale(copy_write, "WRITE_SIZE", mib)
    fd = _per_dispatch(fetch, "FETCH_SIZE")
    wd = _per_dispatch(write, "WRITE_SIZE")
    res = {"fetch_scale": sf, "write_scale": sw, "kernels": {}}
    def match(d, key):
        if key.endswith(","):
            return [v for k, vs in d.items() if k.startswith(key) for v in vs]
        return d.get(key, [])
    for key, (name, srcs) in KERNELS.items():
        f, w = match(fd, key), match(wd, key)
        if not f or not w:
            continue
        fb = sum(f) / len(f) * 1024.0 * sf
        wb = sum(w) / len(w) * 1024.0 * sw
        res["kernels"][name] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb,
                                "dispatches": len(f), "source_sha256": source_hash(srcs)}
    return res


def read_summary(path: str):
    """The JSON record embedded in a summary written by main(), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-json: "):
                return json.loads(line[len("traffic-json: "):])
    return None


def current(record, name):
    """Traffic record of kernel `name` if its sources still match, else None."""
    if not record or name not in record.get("kernels", {}):
        return None
    k = record["kernels"][name]
    if name not in _SOURCES or all(k["source_sha256"] != source_hash(s) for s in _SOURCES[name]):
        return None
    return k


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--copy-fetch", required=True)
    p.add_argument("--copy-write", required=True)
    p.add_argument("--copy-mib", type=int, default=512)
    p.add_argument("--workload", required=True)
    p.add_argument("--command", default="")
    p.add_argument("--out", required=True)
    a = p.parse_args(argv)
    res = summarize(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_mib)
    res["workload"] = a.workload
    lines = [f"# HBM traffic per launch, {a.workload}", "",
             "rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the same counter",
             f"reads for a plain {a.copy_mib} MiB device-to-device copy "
             f"(fetch x{res['fetch_scale']:.3f}, write x{res['write_scale']:.3f}).", ""]
    if a.command:
        lines += ["Commands:", "", "```", a.command, "```", ""]
    lines += ["| kernel | fetch MB | write MB | total MB | dispatches |", "|---|---|---|---|---|"]
    for n, k in res["kernels"].items():
        lines.append(f"| {n} | {k['fetch_bytes'] / 1e6:.1f} | {k['write_bytes'] / 1e6:.1f} | "
                     f"{k['bytes'] / 1e6:.1f} | {k['dispatches']} |")
    lines += ["", "traffic-json: " + json.dumps(res)]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
