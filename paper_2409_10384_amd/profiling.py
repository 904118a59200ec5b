"""Summaries of rocprofv3 output for the committed profile notes.

  python -m paper_2409_10384_amd.profiling stats <kernel_stats.csv>
      per-kernel calls, total and average duration (markdown table)
  python -m paper_2409_10384_amd.profiling traffic <fetch counter_collection.csv>
      <write counter_collection.csv> <out.json>
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel, scaled by what the
      same counters read for the plain copy kernel k_copy of known size
      (1 GiB read + 1 GiB written), written as bytes per launch
"""
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = (1 << 27) * 8

FAMILY_OF_KERNEL = {"k_flux<0>": "flux_x", "k_flux<1>": "flux_y", "k_flux<2>": "flux_z",
                    "k_fofc_flags": "fofc_flags", "k_update": "update", "k_stage_c2p": "stage_c2p",
                    "k_dt": "dt", "k_bcc": "bcc", "k_c2p_batch": "c2p_batch",
                    "k_c2p_learned": "c2p_learned", "k_copy": "copy"}


def short(name):
    """kernel name without namespace, return type and argument list"""
    for k in FAMILY_OF_KERNEL:
        if ("::" + k + "(") in name or name.startswith(k + "("):
            return k
    # 'void (anonymous namespace)::k_emf_edge<1>(...)' -> 'k_emf_edge<1>'
    head = name.replace("(anonymous namespace)", "anon")
    head = head.split("(")[0]
    if "::" in head:
        head = head[head.rindex("::") + 2:]
    return head.split(" ")[-1][:80]


def source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(HERE, "csrc"))):
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stats(path):
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows:
        name = short(r["Name"])
        out.append(f"| {name} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def counter_per_kernel(path, counter):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("Counter-Name", "")) != counter:
            continue
        name = short(r.get("Kernel_Name", r.get("Kernel-Name", "")))
        acc[name].append(float(r.get("Counter_Value", r.get("Counter-Value", 0.0))))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic(fetch_csv, write_csv, out_json):
    fetch = counter_per_kernel(fetch_csv, "FETCH_SIZE")
    write = counter_per_kernel(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (fetch["k_copy"] * 1024.0)
    w_scale = COPY_BYTES / (write["k_copy"] * 1024.0)
    kernels = {}
    for k in fetch:
        fam = FAMILY_OF_KERNEL.get(k)
        if fam is None or fam == "copy":
            continue
        b = fetch[k] * 1024.0 * f_scale + write.get(k, 0.0) * 1024.0 * w_scale
        kernels[fam] = {"kernel": k, "fetch_kib": fetch[k], "write_kib": write.get(k, 0.0),
                        "bytes_per_launch": b}
    d = {"source_hash": source_hash(), "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
         "kernels": kernels}
    json.dump(d, open(out_json, "w"), indent=1)
    return d


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
