"""Full-size oracle runs for the GPU parity tests (test infrastructure).

The FP64 oracle needs tens of seconds per full-size field (the 513^3 field's
Huffman encode dominates), so the GPU test session starts these runs as
child processes as soon as collection is done (see ``conftest.py``) and the
full-size tests wait for their files.  Each job imports only NumPy, the
oracle and the seeded input generators: nothing from the GPU library.

Run one job by hand:  ``python -m tests.oracle_jobs <job> <out_dir>``.

Every job writes ``<out_dir>/<job>.<ext>`` atomically (a temporary name, then
a rename) and, if the oracle raises, ``<out_dir>/<job>.err`` with the
traceback, so a waiting test fails with the oracle's message instead of
timing out.
"""
from __future__ import annotations

import os
import sys
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic  # noqa: E402
from oracle.hierarchy import Hierarchy  # noqa: E402

# The full-size fields (seeded recipes of the benchmark workloads).
FIELDS = {
    "grf513": lambda: synthetic.grf((513, 513, 513), 2),
    "grf300": lambda: synthetic.grf((300, 400, 500), 4),
    "sin8193": lambda: synthetic.sinusoids((8193, 8193), 3),
}

# job name -> (kind, field, norm, relative bound)
STREAM_JOBS = {
    "grf513_linf_1e-3": ("grf513", "linf", 1e-3),
    "grf513_linf_1e-2": ("grf513", "linf", 1e-2),
    "grf513_linf_1e-4": ("grf513", "linf", 1e-4),
    "grf300_linf_1e-4": ("grf300", "linf", 1e-4),
    "grf300_l2_1e-3": ("grf300", "l2", 1e-3),
    "sin8193_linf_1e-4": ("sin8193", "linf", 1e-4),
    "sin8193_l2_1e-3": ("sin8193", "l2", 1e-3),
}
# slices of the 256-array batch (every 8th array, in two halves)
BATCH_JOBS = {"batch256_a": range(0, 128, 8), "batch256_b": range(128, 256, 8)}
TRANSFORM_JOBS = ("grf300_decompose", "grf300_recompose")
ALL_JOBS = tuple(STREAM_JOBS) + tuple(BATCH_JOBS) + TRANSFORM_JOBS


def recompose_input(n: int) -> np.ndarray:
    """Seeded coefficient vector fed to both recompositions."""
    return np.random.default_rng(12).standard_normal(n)


def output_path(out_dir: str, job: str) -> str:
    ext = ".npy" if job in TRANSFORM_JOBS else ".bin"
    return os.path.join(out_dir, job + ext)


def _write_atomic(path: str, writer) -> None:
    tmp = path + ".part"
    with open(tmp, "wb") as f:
        writer(f)
    os.replace(tmp, path)


def run(job: str, out_dir: str) -> None:
    path = output_path(out_dir, job)
    if job in STREAM_JOBS:
        field, norm, rel = STREAM_JOBS[job]
        u = FIELDS[field]()
        blob = oracle.compress(u, rel, norm)
        _write_atomic(path, lambda f: f.write(blob))
    elif job in BATCH_JOBS:
        specs = synthetic.batch_specs(256, seed=5)
        parts = []
        for j in BATCH_JOBS[job]:
            u = synthetic.field_from_spec(specs[j])
            parts.append((j, oracle.compress(u, specs[j]["bound"])))

        def w(f):
            for j, blob in parts:
                f.write(np.asarray([j, len(blob)], dtype="<u8").tobytes())
                f.write(blob)
        _write_atomic(path, w)
    elif job == "grf300_decompose":
        u = FIELDS["grf300"]()
        c = oracle.decompose(u.astype(np.float64), Hierarchy(u.shape))
        _write_atomic(path, lambda f: np.save(f, c))
    elif job == "grf300_recompose":
        h = Hierarchy((300, 400, 500))
        r = oracle.recompose(recompose_input(h.N), h)
        _write_atomic(path, lambda f: np.save(f, r))
    else:
        raise KeyError(job)


def read_batch(path: str) -> dict:
    """{array index: oracle stream bytes} of a batch job's file."""
    data = open(path, "rb").read()
    out, pos = {}, 0
    while pos < len(data):
        j, n = np.frombuffer(data, "<u8", 2, pos)
        pos += 16
        out[int(j)] = data[pos:pos + int(n)]
        pos += int(n)
    return out


if __name__ == "__main__":
    job_name, out = sys.argv[1], sys.argv[2]
    try:
        run(job_name, out)
    except BaseException:
        with open(os.path.join(out, job_name + ".err"), "w") as f:
            f.write(traceback.format_exc())
        raise
