"""Summaries of rocprofv3 output for the committed profile notes.

  python -m paper_2409_10384_amd.profiling stats <kernel_stats.csv>
      per-kernel calls, total and average duration (markdown table)
  python -m paper_2409_10384_amd.profiling fp64 <counter_collection.csv> <out.json> <steps> <tail>
      FP64 lane operations per launch from the four FP64 VALU counters, and per
      RK step over the step's kernels (the run profiled executed <steps> steps; means
      over the last <tail> of them)
  python -m paper_2409_10384_amd.profiling traffic <fetch counter_collection.csv>
      <write counter_collection.csv> <out.json> <steps> <tail>
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


# the sources the kernels of the plain RK step are compiled from (the
# learned inversion, the network and the refined-mesh transfer are not in it)
STEP_SOURCES = ("grmhd.hip", "physics.hpp", "blocks.hpp", "timing.hpp")


def source_hash():
    """hash of the step kernels' sources: counter summaries taken on other
    sources are stale"""
    h = hashlib.sha256()
    for f in STEP_SOURCES:
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


def counter_per_kernel(path, counter, with_count=False, tail=1.0):
    """mean value per dispatch of `counter` for each kernel (and, with
    with_count, the number of dispatches); tail < 1 averages over the last
    fraction `tail` of each kernel's dispatches only (the steady steps after
    the first ones, whose FOFC work is larger)"""
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", r.get("Counter-Name", "")) != counter:
            continue
        name = short(r.get("Kernel_Name", r.get("Kernel-Name", "")))
        did = int(r.get("Dispatch_Id", r.get("Dispatch-Id", len(acc[name]))))
        acc[name].append((did, float(r.get("Counter_Value", r.get("Counter-Value", 0.0)))))
    out = {}
    for k, v in acc.items():
        v.sort()
        m = max(1, int(round(len(v) * tail)))
        vals = [x for _, x in v[-m:]]
        out[k] = (sum(vals) / len(vals), len(v)) if with_count else sum(vals) / len(vals)
    return out


# kernels that run outside the RK step in a profiled bench run (set-up,
# diagnostics, counter calibration)
NOT_IN_STEP = ("k_copy", "k_p2c_block", "k_mass_block", "k_mass_final")


def in_step(kname):
    base = kname.partition("<")[0]
    return base.startswith("k_") and base not in NOT_IN_STEP


def traffic(fetch_csv, write_csv, out_json, steps, tail_steps):
    """scaled HBM bytes per dispatch of every kernel, per family, and summed
    over the kernels of the RK step per step (the profiled run executed
    `steps` steps; per-dispatch means over the last `tail_steps` of them)"""
    tail = tail_steps / steps
    fetch = counter_per_kernel(fetch_csv, "FETCH_SIZE", with_count=True, tail=tail)
    write = counter_per_kernel(write_csv, "WRITE_SIZE", with_count=True, tail=tail)
    f_scale = COPY_BYTES / (fetch["k_copy"][0] * 1024.0)
    w_scale = COPY_BYTES / (write["k_copy"][0] * 1024.0)
    kernels, per_kernel, step_bytes = {}, {}, 0.0
    for k, (fv, n) in fetch.items():
        wv = write.get(k, (0.0, n))[0]
        b = fv * 1024.0 * f_scale + wv * 1024.0 * w_scale
        per_kernel[k] = {"fetch_kib": fv, "write_kib": wv, "bytes_per_dispatch": b, "dispatches": n}
        if in_step(k):
            step_bytes += b * n / steps
        fam = family(k)
        if fam is None or fam == "copy":
            continue
        kernels[fam] = {"kernel": k, "fetch_kib": fv, "write_kib": wv, "bytes_per_launch": b}
    d = {"source_hash": source_hash(), "copy_fetch_scale": f_scale, "copy_write_scale": w_scale,
         "steps": steps, "tail_steps": tail_steps, "bytes_per_step": step_bytes, "kernels": kernels,
         "per_kernel": per_kernel}
    json.dump(d, open(out_json, "w"), indent=1)
    return d


FP64_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_VALU_TRANS_F64")


def fp64(csv_path, out_json, steps, tail_steps):
    """FP64 lane operations per launch of every stage kernel family from one
    pass of the four FP64 VALU instruction counters (wave instructions x 64
    lanes; an FMA counts two operations, a transcendental one), and their sum
    over the kernels of the RK step per step (the profiled run executed
    `steps` steps; per-dispatch means over the last `tail_steps` of them)"""
    tail = tail_steps / steps
    per = {c: counter_per_kernel(csv_path, c, with_count=True, tail=tail) for c in FP64_COUNTERS}
    kernels, per_kernel, step_flops = {}, {}, 0.0
    for k, (_, n) in per["SQ_INSTS_VALU_FMA_F64"].items():
        add, mul, fma, trans = (per[c].get(k, (0.0, n))[0] for c in FP64_COUNTERS)
        fl = 64.0 * (add + mul + 2.0 * fma + trans)
        per_kernel[k] = {"flops_per_dispatch": fl, "dispatches": n}
        if in_step(k):
            step_flops += fl * n / steps
        fam = family(k)
        if fam is None or fam == "copy":
            continue
        kernels[fam] = {"kernel": k, "add": add, "mul": mul, "fma": fma, "trans": trans,
                        "flops_per_launch": fl}
    d = {"source_hash": source_hash(), "steps": steps, "tail_steps": tail_steps,
         "flops_per_step": step_flops, "kernels": kernels, "per_kernel": per_kernel}
    json.dump(d, open(out_json, "w"), indent=1)
    return d


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]),
                                 int(sys.argv[6])), indent=1))
    elif sys.argv[1] == "fp64":
        print(json.dumps(fp64(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5])), indent=1))
