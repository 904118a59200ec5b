"""Summaries of rocprofv3 output for the committed profile notes.

  python -m paper_2409_10384_amd.profiling stats <kernel_stats.csv>
      per-kernel calls, total and average duration (markdown table)
  python -m paper_2409_10384_amd.profiling fp64 <counter_collection.csv> <out.json>
      FP64 lane operations per launch from the four FP64 VALU counters
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

# kernel base name -> timing family; for the per-direction kernels the first
# template argument picks the family
FAMILY_OF_BASE = {"k_fofc_flags": "fofc_flags", "k_fofc_fix": "fofc_fix", "k_update": "update",
                  "k_stage_c2p": "stage_c2p", "k_dt": "dt", "k_bcc": "bcc",
                  "k_c2p_batch": "c2p_batch", "k_c2p_learned": "c2p_learned",
                  "k_stage_c2p_learned": "stage_c2p_learned", "k_mlp_bracket": "mlp_bracket",
                  "k_copy": "copy"}
FLUX_FAMILY = ["flux_x", "flux_y", "flux_z"]


def short(name):
    """kernel name without namespace, return type and argument list, e.g.
    'void (anonymous namespace)::k_flux<1, 0>(...)' -> 'k_flux<1, 0>'"""
    head = name.replace("(anonymous namespace)", "anon")
    depth, cut, start = 0, len(head), 0
    for i, ch in enumerate(head):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif depth == 0 and ch == "(":
            cut = i
            break
        elif depth == 0 and (ch == " " or (ch == ":" and head[i - 1:i] == ":")):
            start = i + 1        # after a top-level space (return type) or '::'
    return head[start:cut][:80]


def family(kname):
    """timing family of a short kernel name (None if not a tracked kernel)"""
    base, _, rest = kname.partition("<")
    args = [a.strip() for a in rest.rstrip(">").split(",")] if rest else []
    if base == "k_flux" and args:
        return FLUX_FAMILY[int(args[0])]
    return FAMILY_OF_BASE.get(base)


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
        fam = family(k)
        if fam is None or fam == "copy":
            continue
        b = fetch[k] * 1024.0 * f_scale + write.get(k, 0.0) * 1024.0 * w_scale
        kernels[fam] = {"kernel": k, "fetch_kib": fetch[k], "write_kib": write.get(k, 0.0),
                        "bytes_per_launch": b}
    d = {"source_hash": source_hash(), "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
         "kernels": kernels}
    json.dump(d, open(out_json, "w"), indent=1)
    return d


FP64_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_VALU_TRANS_F64")


def fp64(csv_path, out_json):
    """FP64 lane operations per launch of every stage kernel family from one
    pass of the four FP64 VALU instruction counters (wave instructions x 64
    lanes; an FMA counts two operations, a transcendental one)"""
    per = {c: counter_per_kernel(csv_path, c) for c in FP64_COUNTERS}
    kernels = {}
    for k in per["SQ_INSTS_VALU_FMA_F64"]:
        fam = family(k)
        if fam is None or fam == "copy":
            continue
        add, mul, fma, trans = (per[c].get(k, 0.0) for c in FP64_COUNTERS)
        kernels[fam] = {"kernel": k, "add": add, "mul": mul, "fma": fma, "trans": trans,
                        "flops_per_launch": 64.0 * (add + mul + 2.0 * fma + trans)}
    d = {"source_hash": source_hash(), "kernels": kernels}
    json.dump(d, open(out_json, "w"), indent=1)
    return d


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
    elif sys.argv[1] == "fp64":
        print(json.dumps(fp64(sys.argv[2], sys.argv[3]), indent=1))
