"""Tune tables that force one GEMM-1 choice on every supernode (tests)."""

import json
import os
import tempfile

S_BUCKETS = (16, 64, 128, 256)
C_BUCKETS = (64, 256, 1024, 4096, 1 << 30)
FORCED = {
    "dense_ydense": {"dense": 1, "ydense": 1},
    "dense_fused": {"dense": 1, "ydense": 0},
    "gather": {"dense": 0, "ydense": 0},
    "dense_ydense128": {"dense": 1, "ydense": 1, "tile": 128},
}


def key():
    from paper_1604_02528_amd import capi

    return dict(kv.split("=") for kv in capi.selinv_tune_key().split())


def forced_table(choice, dtype, split_min_k=0, arch=None, rocm=None):
    """Path of a temporary table giving `choice` to every bucket of `dtype`."""
    k = key()
    entries = [dict(arch=arch or k["arch"], rocm=rocm or k["rocm"], dtype=dtype, s_max=s, c_max=c,
                    split_min_k=split_min_k, **FORCED[choice]) for s in S_BUCKETS for c in C_BUCKETS]
    f = tempfile.NamedTemporaryFile("w", suffix=".json", delete=False)
    json.dump({"format": "selinv-tune-1", "entries": entries}, f)
    f.close()
    return f.name


def remove(path):
    try:
        os.unlink(path)
    except OSError:
        pass
