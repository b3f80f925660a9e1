"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1602_03395_amd.profiling stats <kernel_stats.csv>
        markdown table of per-kernel call counts and durations
    python -m paper_1602_03395_amd.profiling counters <counter_collection.csv> <COUNTER>
        average counter value per dispatch for every kernel name
    python -m paper_1602_03395_amd.profiling traffic <fetch.csv> <write.csv> <copy_MiB> <calls> <out.json> <tag>
        HBM bytes per dispatch of every pass of the schedule (key 'kind#ordinal', ordinal counted
        within one expansion call; <calls> = expansion calls in the profiled run) from FETCH_SIZE
        and WRITE_SIZE (KiB per dispatch), each scaled by the factor that makes the plain copy
        kernel of known size read (and write) exactly its size; stored under <tag>
        (workload/dtype/schedule) and stamped with the hash of the kernel sources

    python -m paper_1602_03395_amd.profiling traffic-kernels <fetch.csv> <write.csv> <copy_MiB> <out.json> <tag>
                                                   <kernel=key> ...
        the same per kernel name (runs whose passes interleave over several streams), stored
        under the given keys

    python -m paper_1602_03395_amd.profiling passes <kernel_trace.csv> <calls>
        markdown table of the average kernel-trace duration of every pass of the schedule (key
        'kind#ordinal' as above; <calls> = expansion calls in the traced run)

Only the csv files rocprofv3 writes are read; nothing here touches the GPU.
"""

from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def short_name(name: str) -> str:
    """fx::k_EA<float, 8>(...) -> k_EA<float,8>; other kernels keep a trimmed name."""
    m = re.search(r"(k_[A-Za-z0-9]+<[^>]*>)", name)
    if m:
        return m.group(1).replace(" ", "")
    return name.split("(")[0][-80:]


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| %s | %s | %.3f | %.2f | %.1f |" % (
            short_name(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def copy_counter(path: str, counter: str):
    """(kernel name, value) of the calibration copy: the largest single dispatch of a copy kernel
    (other copies in the run, such as uploads of inputs, are smaller)."""
    best = None
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter or "copy" not in r["Kernel_Name"].lower():
            continue
        v = float(r["Counter_Value"])
        if best is None or v > best[1]:
            best = (r["Kernel_Name"], v)
    if best is None:
        raise SystemExit("no copy kernel found in the counter file")
    return best


def counters(path: str, counter: str):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


KERNEL_SOURCES = ("kernels.hip", "kernels_p2.hip", "kernels_ct.hip", "kernels_cfp.hip", "device_common.h",
                  "fx_internal.h")


def code_lines(text: str):
    """The lines of a source with its // comments, trailing blanks and empty lines dropped."""
    for line in text.splitlines():
        line = line.split("//", 1)[0].rstrip()
        if line:
            yield line


def kernels_hash(sources: dict | None = None) -> str:
    """Hash of the code of the kernel sources (files under csrc/, or the given name -> text), with
    comments and all white space removed: an edit of comments or layout alone leaves it, and so
    the stored counters, valid."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        if sources is not None:
            text = sources[name]
        else:
            with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as f:
                text = f.read()
        code = "".join("".join(line.split()) for line in code_lines(text))
        h.update(name.encode("utf-8") + b"\0" + code.encode("utf-8") + b"\0")
    return h.hexdigest()[:16]


# pass kernels: k_E, k_E2 (power-of-two), k_Ect (3*2^k), k_ER / k_ERW / k_ERG (register forms), k_EA*,
# k_EAW, k_A, k_AS / k_ASR / k_ASK (structured accumulates), k_AA (fused two-axis accumulate), adjoints
# (k_EH*, k_EHG, k_AH*)
PASS_KIND = re.compile(r"\bk_(EAH|EA|EH|AH|AAH|AA|E|A)(?:2|ct|S|R|SR|SK|RW|RG|W|G)?<")


def pass_kind(name: str):
    """Kind of the pass a kernel name runs (E, EA, A, AA, EH, AH, ...), or None. k_ERG serves E and
    EA; its last template argument tells them apart."""
    m = PASS_KIND.search(name)
    if not m:
        return None
    if "k_ERG<" in name and re.search(r"k_ERG<[^>]*,\s*true\s*>", name):
        return "EA"
    return m.group(1)


def _pass_dispatches(path: str, counter: str):
    """[(dispatch_id, kind, value)] of the pass kernels, in dispatch order."""
    out = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        kind = pass_kind(r["Kernel_Name"])
        if kind:
            out.append((int(r["Dispatch_Id"]), kind, float(r["Counter_Value"])))
    out.sort()
    return out


def _per_pass(rows, calls_per_run: int):
    """Average value per (kind, ordinal within one expansion call); key 'kind#ordinal'."""
    by_kind = collections.defaultdict(list)
    for _, kind, v in rows:
        by_kind[kind].append(v)
    res = {}
    for kind, vals in by_kind.items():
        per_call = max(1, len(vals) // max(1, calls_per_run))
        for i, v in enumerate(vals):
            key = f"{kind}#{i % per_call}"
            res.setdefault(key, []).append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in res.items()}


def traffic(fetch_csv: str, write_csv: str, copy_mib: float, calls: int, out_json: str, tag: str):
    copy_kib = copy_mib * 1024.0
    ck, cf = copy_counter(fetch_csv, "FETCH_SIZE")
    _, cw = copy_counter(write_csv, "WRITE_SIZE")
    f_scale = copy_kib / cf
    w_scale = copy_kib / cw
    fp = _per_pass(_pass_dispatches(fetch_csv, "FETCH_SIZE"), calls)
    wp = _per_pass(_pass_dispatches(write_csv, "WRITE_SIZE"), calls)
    res = {"copy_kernel": short_name(ck), "copy_MiB": copy_mib,
           "copy_fetch_KiB_counter": cf, "copy_write_KiB_counter": cw,
           "fetch_scale": f_scale, "write_scale": w_scale, "passes": {}}
    for key, (fv, n) in fp.items():
        fb = fv * 1024.0 * f_scale
        wb = wp.get(key, (0.0, 0))[0] * 1024.0 * w_scale
        res["passes"][key] = {"dispatches": n, "fetch_bytes": fb, "write_bytes": wb,
                              "hbm_bytes_per_launch": fb + wb}
    _store(out_json, tag, res)
    return res


def _store(out_json: str, tag: str, res: dict):
    doc = {}
    if os.path.exists(out_json):
        try:
            doc = json.load(open(out_json))
        except ValueError:
            doc = {}
    if doc.get("kernels_hash") != kernels_hash():
        doc = {"kernels_hash": kernels_hash(), "workloads": {}}
    doc.setdefault("workloads", {})[tag] = res
    json.dump(doc, open(out_json, "w"), indent=1)


def strided_calibration(fetch_csv: str, write_csv: str, copy_mib: float, f_scale: float, w_scale: float):
    """Check of the copy factors on partial-line reads: the benchmark's calibration follows the plain
    copy with two strided gathers of the same source, viewed as rows of 512 bytes, keeping the first
    256 bytes of every row, then the first 64 (the first two copy dispatches that are not runtime
    blits, in dispatch order). Returns raw and scaled counters against the bytes each gather moves."""
    def gathers(path, counter):
        rows = []
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if r.get("Counter_Name") != counter or "copy" not in name.lower() or "rocclr" in name.lower():
                continue
            rows.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        rows.sort()
        return [v for _, v in rows[:2]]

    fg, wg = gathers(fetch_csv, "FETCH_SIZE"), gathers(write_csv, "WRITE_SIZE")
    out = []
    for i, (frac, run) in enumerate(((0.5, 256), (0.125, 64))):
        if i >= len(fg) or i >= len(wg):
            break
        kib = copy_mib * 1024.0 * frac
        out.append({"run_bytes": run, "row_bytes": 512, "moved_KiB_each_way": kib,
                    "fetch_KiB_counter": fg[i], "write_KiB_counter": wg[i],
                    "fetch_scaled_over_moved": fg[i] * f_scale / kib,
                    "write_scaled_over_moved": wg[i] * w_scale / kib})
    return out


def traffic_kernels(fetch_csv: str, write_csv: str, copy_mib: float, out_json: str, tag: str, mapping,
                    bench_json: str = None):
    """As ``traffic``, but per kernel name (for runs whose passes interleave, such as a batch whose
    classes run on several streams): ``mapping`` is a list of 'short_name=key' (the key under which
    the bench looks the kernel up, e.g. '64x64x512/EA#0'); bytes are averages per dispatch. With
    ``bench_json`` (the benchmark line of the same launch configuration) every entry also records
    the item shape of its launches and the ratio of measured to algorithmic bytes."""
    rows = {}
    if bench_json:
        line = [ln for ln in open(bench_json).read().splitlines() if ln.strip().startswith("{")][-1]
        for r in json.loads(line).get("passes", []):
            rows[f'{r["class"]}/{r["key"]}'] = r
    f_avg, f_n = counters(fetch_csv, "FETCH_SIZE")
    w_avg, _ = counters(write_csv, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    ck, cf = copy_counter(fetch_csv, "FETCH_SIZE")
    _, cw = copy_counter(write_csv, "WRITE_SIZE")
    f_scale = copy_kib / cf
    w_scale = copy_kib / cw
    res = {"copy_kernel": short_name(ck), "copy_MiB": copy_mib,
           "copy_fetch_KiB_counter": cf, "copy_write_KiB_counter": cw,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "strided_check": strided_calibration(fetch_csv, write_csv, copy_mib, f_scale, w_scale), "passes": {}}
    by_short = {short_name(k): k for k in f_avg}
    for item in mapping:
        name, key = item.split("=", 1)
        full = by_short.get(name)
        if full is None:
            raise SystemExit(f"kernel {name} not in the counter file")
        fb = f_avg[full] * 1024.0 * f_scale
        wb = w_avg.get(full, 0.0) * 1024.0 * w_scale
        ent = {"kernel": name, "dispatches": f_n[full], "fetch_KiB_counter": f_avg[full],
               "write_KiB_counter": w_avg.get(full, 0.0), "fetch_bytes": fb, "write_bytes": wb,
               "hbm_bytes_per_launch": fb + wb}
        r = rows.get(key)
        if r:
            alg = r["bytes"] / r["launches"]
            ent.update({"group": r["group"], "q_block": r["q_block"], "algorithmic_bytes_per_launch": alg,
                        "traffic_over_algorithmic": (fb + wb) / alg})
        res["passes"][key] = ent
    _store(out_json, tag, res)
    return res


def passes(trace_csv: str, calls: int) -> str:
    rows = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
                  for r in csv.DictReader(open(trace_csv)))
    seq = [(k, (e - b) / 1e3) for b, e, n in rows for k in [pass_kind(n)] if k]
    per = max(1, len(seq) // max(1, calls))
    kinds = [k for k, _ in seq[:per]]
    acc = collections.OrderedDict()
    for i, (kind, us) in enumerate(seq):
        j = i % per
        acc.setdefault(f"{kind}#{kinds[:j].count(kind)}", []).append(us)
    out = ["| pass | launches | avg us |", "|---|---:|---:|"]
    out += ["| %s | %d | %.2f |" % (k, len(v), sum(v) / len(v)) for k, v in acc.items()]
    return "\n".join(out)


def phases(trace_csv: str, kernel: str, per_run: int, labels):
    """Average duration (us) of one kernel's dispatches per run, counted from the end of the trace:
    the last per_run dispatches belong to labels[-1], the per_run before them to labels[-2], ...; a
    label "name*k" covers k runs. What precedes them is reported as "earlier"."""
    d = sorted((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
               for r in csv.DictReader(open(trace_csv)) if short_name(r["Kernel_Name"]) == kernel)
    durs = [x for _, x in d]
    out = ["| dispatches | runs | avg us |", "|---|---:|---:|"]
    end = len(durs)
    rows = []
    for lab in reversed(labels):
        name, _, k = lab.partition("*")
        k = int(k) if k else 1
        seg = durs[max(0, end - k * per_run):end]
        end -= len(seg)
        if seg:
            rows.append("| %s | %d | %.1f |" % (name, k, sum(seg) / len(seg)))
    if end > 0:
        rows.append("| earlier (set-up) | | %.1f |" % (sum(durs[:end]) / end))
    return "\n".join(out + list(reversed(rows)))


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "stats":
        print(stats(sys.argv[2]))
    elif cmd == "phases":
        print(phases(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5:]))
    elif cmd == "passes":
        print(passes(sys.argv[2], int(sys.argv[3])))
    elif cmd == "counters":
        avg, n = counters(sys.argv[2], sys.argv[3])
        for k in sorted(avg, key=lambda x: -avg[x]):
            print(f"{short_name(k):40s} dispatches {n[k]:5d}  avg {avg[k]:.4g}")
    elif cmd == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), int(sys.argv[5]), sys.argv[6],
                                 sys.argv[7]), indent=1))
    elif cmd == "traffic-kernels":
        rest = sys.argv[7:]
        bench = None
        if rest and rest[0].startswith("--bench="):
            bench, rest = rest[0].split("=", 1)[1], rest[1:]
        print(json.dumps(traffic_kernels(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6],
                                         rest, bench), indent=1))
    else:
        raise SystemExit(__doc__)
