"""HBM traffic of the dominant kernel from hardware counters.

Two counter passes of the same short bench run (each its own rocprofv3
process), FETCH_SIZE and WRITE_SIZE in KiB per dispatch, are scaled by what the
same counters read for the plain copy kernel of known size that the run also
launches (bench.py --copy-probe-mib).  The result is stored in counters.json
next to this file together with a hash of the kernel's sources; bench.py reports
it only while the sources still match (otherwise the counters describe a kernel
that no longer exists and the traffic is reported as null).

Usage, from the repository root (cd /tmp && export TMPDIR=/tmp first):

  rocprofv3 --pmc FETCH_SIZE -d OUT/pmc_fetch -o run -- python <repo>/bench.py \\
      --steps 6 --warmup 2 --profile-steps 2 --no-cpu-baseline --no-fp64 --no-serve --copy-probe-mib 1024
  rocprofv3 --pmc WRITE_SIZE -d OUT/pmc_write -o run -- python <repo>/bench.py (same flags)
  python -m paper_1607_04572_amd.counters OUT/pmc_fetch/run_results.db OUT/pmc_write/run_results.db 1024

The FP32 EK kernel is bound by its vector ALU work, not by HBM: its VALU
instruction count per launch comes from an SQ counter pass of the same run
(SQ_INSTS_VALU with SQ_WAVES), stored in counters_valu.json with a hash of the
EK sources:

  rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU -d OUT/pmc_sq -o run -- python <repo>/bench.py (same flags)
  python -m paper_1607_04572_amd.counters --valu OUT/pmc_sq/run_results.db
"""
from __future__ import annotations

import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STORE = os.path.join(HERE, "counters.json")
KERNEL = "k_lb<float, true>"
SOURCES = ["csrc/ek_lb.h", "csrc/ek_lb.hip", "csrc/ek_internal.h"]
# Kernels of one FP32 step (k_move runs apart only at the start of a graph-replayed chain of steps, with
# no measurable traffic), for the step-level figure; it holds while no kernel source has changed.
STEP_KERNELS = ["k_lb<float", "k_ek32<", "k_fft_", "k_geometry<float", "k_boundary<float", "k_boundary_post<float",
                "k_pool<float", "k_particle_forces<float", "k_finish<float"]


VALU_STORE = os.path.join(HERE, "counters_valu.json")
EK_KERNEL = "k_ek32<"
EK_SOURCES = ["csrc/ek_fields.hip", "csrc/ek_lb.h", "csrc/ek_internal.h"]


def source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for s in sources or SOURCES:
        with open(os.path.join(HERE, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def all_sources() -> list:
    d = os.path.join(HERE, "csrc")
    return sorted("csrc/" + f for f in os.listdir(d) if f.endswith((".h", ".hip", ".cpp")))


def per_dispatch(db: str, counter: str) -> dict:
    """Mean value of one counter per kernel (summed over instances of a dispatch)."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id", (counter,)).fetchall()
    acc: dict = {}
    for name, _, v in rows:
        acc.setdefault(name, []).append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def pick(d: dict, key: str) -> float:
    hits = [v for k, v in d.items() if key in k]
    if not hits:
        raise KeyError(f"no dispatch of {key} in the counter data")
    return hits[0]


def main(fetch_db: str, write_db: str, copy_mib: int) -> dict:
    fetch = per_dispatch(fetch_db, "FETCH_SIZE")
    write = per_dispatch(write_db, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    f_copy, w_copy = pick(fetch, "k_copy16"), pick(write, "k_copy16")
    f_scale, w_scale = copy_kib / f_copy, copy_kib / w_copy
    f_lb, w_lb = pick(fetch, KERNEL), pick(write, KERNEL)
    out = {
        "kernel": KERNEL,
        "source_sha256": source_hash(),
        "fetch_kib_per_dispatch": f_lb, "write_kib_per_dispatch": w_lb,
        "copy_probe_mib": copy_mib, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "traffic_bytes_per_launch": (f_lb * f_scale + w_lb * w_scale) * 1024.0,
        "read_bytes_per_launch": f_lb * f_scale * 1024.0, "write_bytes_per_launch": w_lb * w_scale * 1024.0,
        "all_kernels_fetch_kib": fetch, "all_kernels_write_kib": write,
        "step_bytes": sum(fetch[k] * f_scale * 1024.0 + write.get(k, 0.0) * w_scale * 1024.0
                          for k in fetch if any(s in k for s in STEP_KERNELS)),
        "all_sources_sha256": source_hash(all_sources()),
    }
    with open(STORE, "w") as f:
        json.dump(out, f, indent=1)
    return out


def stored_step_bytes() -> float | None:
    """HBM bytes of one FP32 step from the stored passes, if no kernel source has changed since."""
    if not os.path.exists(STORE):
        return None
    with open(STORE) as f:
        d = json.load(f)
    return d.get("step_bytes") if d.get("all_sources_sha256") == source_hash(all_sources()) else None


def stored_traffic() -> dict | None:
    """The stored measurement if it describes the current sources, else None."""
    if not os.path.exists(STORE):
        return None
    with open(STORE) as f:
        d = json.load(f)
    return d if d.get("source_sha256") == source_hash() else None


def store_valu(sq_db: str) -> dict:
    """VALU instructions (wave64 instructions issued, all waves) and waves per launch of the FP32 EK kernel."""
    valu = per_dispatch(sq_db, "SQ_INSTS_VALU")
    waves = per_dispatch(sq_db, "SQ_WAVES")
    out = {"kernel": EK_KERNEL, "source_sha256": source_hash(EK_SOURCES),
           "valu_per_launch": pick(valu, EK_KERNEL), "waves_per_launch": pick(waves, EK_KERNEL)}
    with open(VALU_STORE, "w") as f:
        json.dump(out, f, indent=1)
    return out


def stored_valu() -> dict | None:
    """The stored EK instruction count if it describes the current EK sources, else None."""
    if not os.path.exists(VALU_STORE):
        return None
    with open(VALU_STORE) as f:
        d = json.load(f)
    return d if d.get("source_sha256") == source_hash(EK_SOURCES) else None


if __name__ == "__main__":
    if sys.argv[1] == "--valu":
        print(json.dumps(store_valu(sys.argv[2]), indent=1))
    else:
        r = main(sys.argv[1], sys.argv[2], int(sys.argv[3]))
        print(json.dumps({k: v for k, v in r.items() if not k.startswith("all_")}, indent=1))
