"""Summarise rocprofv3 results of a bench.py run into per-kernel and per-family tables.

Reads the SQLite result files that rocprofv3 writes (`<dir>/<name>_results.db`):

* a kernel-trace run (`--kernel-trace --stats`): dispatch count, total and average
  duration per kernel symbol and per kernel family;
* optionally a `--pmc FETCH_SIZE` run and a `--pmc WRITE_SIZE` run of the same command:
  HBM bytes per dispatch, calibrated against a device copy of known size that the
  command performs (bench.py --calib-copy-gib), and the ratio of measured to
  algorithmic bytes per family.

Only the dispatches between the two marker kernels that bench.py launches around its
timed region (a one-element uint8 fill before and after) are counted, so the launch mix
is that of the timed steps.  The family byte models are the ones the library uses for
its live accounting (mesh r = 4 Ng^3 bytes, half spectrum c = 8 Ng^2 (Ng/2+1), P
particles).

    python -m paper_2211_09958_amd.rocprof_summary --kt DIR/kt_results.db \
        [--fetch DB --write DB] --ptcl 512 --mesh 1024 --workload NAME --out DIR \
        --command-kt "..." [--command-fetch "..." --command-write "..."]
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
MARKER = "FillFunctor<unsigned char>"
CALIB = "__amd_rocclr_copyBuffer"


FFT_SOURCES = ("fft.hip", "fft_engine.h", "fft_plan.h", "layout.h", "xcd.h")
PARTICLE_SOURCES = ("particles.hip", "layout.h", "xcd.h")
FAMILY_SOURCES = {"fft_x": FFT_SOURCES, "fft_strided": FFT_SOURCES, "grad_z": FFT_SOURCES,
                  "grad_adj_z": FFT_SOURCES, "scatter": PARTICLE_SOURCES,
                  "scatter_vec": PARTICLE_SOURCES, "gather": PARTICLE_SOURCES,
                  "unkick_vjp": PARTICLE_SOURCES, "wgrad": PARTICLE_SOURCES,
                  "bin": PARTICLE_SOURCES}


# C/C++ comments, and the string and character literals that may contain comment markers
_CODE_TOKENS = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'', re.S)


def code_only(text: str) -> str:
    """Source text without comments and blank lines, trailing blanks stripped: what the
    compiler sees, for deciding whether kernels changed."""
    text = _CODE_TOKENS.sub(lambda m: "" if m.group(0).startswith("/") else m.group(0), text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def sources_sha256(family: str) -> str:
    """Hash of the kernel sources (kernels and their launchers) of a family, comments and
    blank lines left out; its counter figures go stale when it changes."""
    h = hashlib.sha256()
    for name in FAMILY_SOURCES[family]:
        h.update(name.encode())
        with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("pmx::", "")
    n = re.sub(r"^void ", "", n)
    depth, out = 0, []
    for ch in n:          # drop the parameter list, keep template arguments
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).strip()


def family(sym: str, ng: int):
    """(family, algorithmic-bytes rule) of a kernel symbol, or (None, None)."""
    m = re.match(r"(k_\w+)(?:<([^>]*)>)?", sym)
    if not m:
        return None, None
    base, targs = m.group(1), [t.strip() for t in (m.group(2) or "").split(",") if t.strip()]
    if base in ("k_fft_x_r2c", "k_fft_x_c2r") and targs[:1] == [str(ng)]:
        return "fft_x", "rc_per_buf"
    if base == "k_fft_strided" and targs[:1] == [str(ng)]:
        return "fft_strided", "2c_per_buf"
    if base in ("k_fft_y_split", "k_fft_y_merge") and targs[:1] == [str(ng)]:
        return "fft_strided", "3c"
    if base in ("k_grad_z", "k_grad_z_pipe") and targs[:1] == [str(ng)]:
        return "grad_z", "3c"
    if base in ("k_grad_adj_z", "k_grad_adj_z_pipe") and targs[:1] == [str(ng)]:
        return "grad_adj_z", "4c" if targs[1:] == ["true"] else "3c"
    if base == "k_scatter_tile":
        return ("scatter_vec", "24P+3r") if targs[1:] == ["true"] else ("scatter", "12P+r")
    if base == "k_gather_tile":
        mode = targs[1] if len(targs) > 1 else ""
        # kick-drift and un-drift gathers also write each moved particle's bin key
        # and rank (8 bytes) for the next sort
        return {"0": ("gather", "56P+3r"), "1": ("gather", "24P+3r"),
                "2": ("unkick_vjp", "72P+3r"), "3": ("wgrad", "92P+r")}.get(mode, (None, None))
    if base in ("k_bin_count", "k_scan_local", "k_scan_bsum", "k_scan_add", "k_index",
                "k_compact_sorted"):
        return "bin", None
    if base.startswith("k_mlp") or base == "k_adam":
        return "mlp", None
    return None, None


def alg_bytes(rule, grid_y, P, ng):
    r = 4.0 * ng ** 3
    c = 8.0 * ng * ng * (ng // 2 + 1)
    return {"rc_per_buf": grid_y * (r + c), "2c_per_buf": grid_y * 2 * c, "3c": 3 * c, "4c": 4 * c,
            "5c": 5 * c, "24P+3r": 24 * P + 3 * r, "12P+r": 12 * P + r,
            "56P+3r": 56 * P + 3 * r,
            "72P+3r": 72 * P + 3 * r, "92P+r": 92 * P + r}.get(rule)


def dispatches(db: str, counter: str | None = None):
    """[(dispatch_id, name, grid_y, duration_ns, counter_value)] in dispatch order."""
    con = sqlite3.connect(db)
    if counter is None:
        rows = con.execute("select dispatch_id, name, grid_y, duration, 0.0 from kernels "
                           "order by dispatch_id").fetchall()
    else:
        rows = con.execute(
            "select k.dispatch_id, k.name, k.grid_y, k.duration, e.counter_value "
            "from pmc_events e join kernels k on e.dispatch_id = k.dispatch_id "
            "where e.counter_name = ? order by k.dispatch_id", (counter,)).fetchall()
    con.close()
    return rows


RESOURCE_COLUMNS = (("VGPRs", ("arch_vgpr_count", "vgpr_count")),
                    ("AGPRs", ("accum_vgpr_count", "agpr_count")),
                    ("SGPRs", ("sgpr_count",)),
                    ("LDS bytes", ("group_segment_size", "lds_size", "lds_block_size")),
                    ("scratch bytes", ("private_segment_size", "scratch_size")),
                    ("work-group", ("workgroup_size",)))


def resources(db: str):
    """{kernel name: [(column label, value)]} from the per-dispatch resource columns
    that the kernel trace records (register counts, LDS and scratch per work-group);
    the column names differ between rocprofv3 versions, so they are looked up."""
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(kernels)").fetchall()]
    picked = []
    for label, names in RESOURCE_COLUMNS:
        for n in names:
            if n in cols:
                picked.append((label, n))
                break
    if "workgroup_size" not in cols and {"workgroup_x", "workgroup_y", "workgroup_z"} <= set(cols):
        picked.append(("work-group", "workgroup_x * workgroup_y * workgroup_z"))
    out = {}
    if picked:
        q = "select name, " + ", ".join(c for _, c in picked) + " from kernels group by name"
        for row in con.execute(q).fetchall():
            out[row[0]] = [(label, v) for (label, _), v in zip(picked, row[1:])]
    con.close()
    return out


def timed_window(rows):
    """Rows strictly between the first two marker dispatches (all rows if absent)."""
    idx = [i for i, r in enumerate(rows) if MARKER in r[1]]
    if len(idx) >= 2:
        return rows[idx[0] + 1: idx[1]], True
    return rows, False


def calibration(rows, calib_bytes):
    """Factor true/read of a counter, from the device copy of calib_bytes that bench.py
    issues just before its first marker (the last copy dispatch ahead of it)."""
    first = next((i for i, r in enumerate(rows) if MARKER in r[1]), len(rows))
    cand = [r for r in rows[:first] if r[1] == CALIB]
    if not cand or calib_bytes <= 0 or cand[-1][4] <= 0:
        return None
    return calib_bytes / (cand[-1][4] * 1024.0), cand[-1][0]


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--ptcl", type=int, required=True)
    ap.add_argument("--mesh", type=int, required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--calib-bytes", type=float, default=float(2 ** 30))
    ap.add_argument("--out", required=True)
    ap.add_argument("--command-kt", default="")
    ap.add_argument("--command-fetch", default="")
    ap.add_argument("--command-write", default="")
    a = ap.parse_args()
    P, ng = a.ptcl ** 3, a.mesh
    os.makedirs(a.out, exist_ok=True)

    rows, marked = timed_window(dispatches(a.kt))
    per_sym = collections.OrderedDict()
    per_fam = collections.defaultdict(lambda: [0, 0.0])
    for _, name, gy, dur, _ in rows:
        s = short(name)
        e = per_sym.setdefault(s, [0, 0.0])
        e[0] += 1
        e[1] += dur
        fam, _ = family(s, ng)
        if fam:
            per_fam[fam][0] += 1
            per_fam[fam][1] += dur
    total = sum(v[1] for v in per_sym.values())
    summarised = "python -m paper_2211_09958_amd.rocprof_summary " + " ".join(
        f"'{x}'" if " " in x else x for x in sys.argv[1:])
    lines = [f"# rocprofv3 kernel trace: {a.workload}", "",
             f"Command (from the repository root): `{a.command_kt}`", "",
             f"Summarised with: `{summarised}`", "",
             f"Window: {'dispatches between the timed-region markers' if marked else 'whole run'}"
             f"; {len(rows)} dispatches, {total / 1e6:.1f} ms of kernel time.", "",
             "## Per family (library kernel families)", "",
             "| family | dispatches | total ms | avg ms / dispatch |", "|---|---|---|---|"]
    for fam, (n, t) in sorted(per_fam.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {fam} | {n} | {t / 1e6:.2f} | {t / n / 1e6:.4f} |")
    lines += ["", "## Per kernel symbol", "", "| kernel | calls | total ms | avg ms | % |",
              "|---|---|---|---|---|"]
    for s, (n, t) in sorted(per_sym.items(), key=lambda kv: -kv[1][1]):
        if t / total < 1e-4:
            continue
        lines.append(f"| `{s}` | {n} | {t / 1e6:.2f} | {t / n / 1e6:.4f} | {100 * t / total:.2f} |")
    res = {short(k): v for k, v in resources(a.kt).items()}
    shown = [s for s, (n, t) in sorted(per_sym.items(), key=lambda kv: -kv[1][1])
             if t / total >= 1e-4 and s in res]
    if shown:
        labels = [label for label, _ in res[shown[0]]]
        lines += ["", "## Per kernel symbol: resources (from the kernel trace)", "",
                  "Register counts as the trace records them; for these wave64 kernels its "
                  "VGPR figure is half the `.vgpr_count` of the code object's metadata (for "
                  "example 249 for `k_grad_z_pipe<1024>`, recorded as 128): waves per SIMD = "
                  "512 / (2 x VGPRs), at most 8.", "",
                  "| kernel | " + " | ".join(labels) + " |",
                  "|---|" + "---|" * len(labels)]
        for s in shown:
            lines.append(f"| `{s}` | " + " | ".join(str(v) for _, v in res[s]) + " |")
    tag = a.workload
    with open(os.path.join(a.out, f"kernel-trace_all-kernels_{tag}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    if not (a.fetch and a.write):
        return
    frows_all = dispatches(a.fetch, "FETCH_SIZE")
    wrows_all = dispatches(a.write, "WRITE_SIZE")
    fcal = calibration(frows_all, a.calib_bytes)
    wcal = calibration(wrows_all, a.calib_bytes)
    if not (fcal and wcal):
        raise SystemExit("no calibration copy before the first marker (run bench.py with "
                         "--calib-copy-gib)")
    ff, wf = fcal[0], wcal[0]
    frows, _ = timed_window(frows_all)
    wrows, _ = timed_window(wrows_all)
    wmap = {r[0]: r[4] for r in wrows}
    groups = collections.OrderedDict()
    fam_tot = collections.defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    for did, name, gy, _, fv in frows:
        s = short(name)
        wv = wmap.get(did)
        if wv is None:
            continue
        key = (s, gy)
        g = groups.setdefault(key, [0, 0.0, 0.0])
        g[0] += 1
        g[1] += fv * 1024.0 * ff
        g[2] += wv * 1024.0 * wf
        fam, rule = family(s, ng)
        if fam and rule:
            ab = alg_bytes(rule, gy, P, ng)
            t = fam_tot[fam]
            t[0] += 1
            t[1] += fv * 1024.0 * ff
            t[2] += wv * 1024.0 * wf
            t[3] += ab
    lines = [f"# rocprofv3 HBM traffic (FETCH_SIZE, WRITE_SIZE): {a.workload}", "",
             f"FETCH_SIZE command (from the repository root): `{a.command_fetch}`", "",
             f"WRITE_SIZE command: `{a.command_write}`", "",
             f"Summarised with: `{summarised}`", "",
             f"Calibration: a device copy of {a.calib_bytes / 2 ** 30:g} GiB reads "
             f"FETCH_SIZE = {1 / ff:.3f}x and WRITE_SIZE = {1 / wf:.3f}x its true bytes; "
             f"counter values are multiplied by {ff:.3f} (fetch) and {wf:.3f} (write).", "",
             "## Per family: measured vs algorithmic bytes per dispatch", "",
             "| family | dispatches | fetch GB/disp | write GB/disp | measured GB/disp | "
             "algorithmic GB/disp | measured / algorithmic |", "|---|---|---|---|---|---|---|"]
    traffic = {"workload": a.workload,
               "fetch_factor": ff, "write_factor": wf, "families": {}}
    for fam, (n, fb, wb, ab) in sorted(fam_tot.items(), key=lambda kv: -kv[1][3]):
        ratio = (fb + wb) / ab if ab else None
        lines.append(f"| {fam} | {n} | {fb / n / 1e9:.3f} | {wb / n / 1e9:.3f} | "
                     f"{(fb + wb) / n / 1e9:.3f} | {ab / n / 1e9:.3f} | {ratio:.3f} |")
        traffic["families"][fam] = {"sources_sha256": sources_sha256(fam),
                                    "dispatches": n, "measured_bytes_per_dispatch": (fb + wb) / n,
                                    "algorithmic_bytes_per_dispatch": ab / n,
                                    "measured_over_algorithmic": ratio}
    lines += ["", "## Per kernel symbol and grid_y (buffers per launch)", "",
              "| kernel | grid_y | dispatches | fetch MB/disp | write MB/disp |",
              "|---|---|---|---|---|"]
    for (s, gy), (n, fb, wb) in sorted(groups.items(), key=lambda kv: -(kv[1][1] + kv[1][2])):
        if (fb + wb) / n < 1e6:
            continue
        lines.append(f"| `{s}` | {gy} | {n} | {fb / n / 1e6:.1f} | {wb / n / 1e6:.1f} |")
    with open(os.path.join(a.out, f"hbm-traffic_all-kernels_{tag}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(a.out, "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1)


if __name__ == "__main__":
    main()
