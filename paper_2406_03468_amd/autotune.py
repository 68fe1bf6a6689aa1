"""A JSON cache of fused-pass tunings (``fs_tune_pass``), keyed by (arch, n, floor(log2 m), dtype).

``tune`` times the admissible (tile height H, work-group count G) pairs of the fused pass over A
through the library, keeps the fastest in the context and records it in the cache; ``apply`` loads
every entry of one architecture into a context (``fs_set_pass_tuning``), so later solves of those
shapes use the tuned pass without timing again.  The file is plain JSON:
``{"gfx950|1000|19|f64": {"H": 16, "G": 256, "ms": 1.3}, ...}``.  The timing itself runs in the
library; this module only keeps the table.
"""

import json
import os

from . import binding


def m_bucket(m: int) -> int:
    """floor(log2 m), the library's key for the row count."""
    return int(m).bit_length() - 1


def key(arch: str, n: int, m: int, dtype: str = "f64") -> str:
    return f"{arch}|{int(n)}|{m_bucket(m)}|{dtype}"


def device_arch(device: int = 0) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def load(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(cache: dict, path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx, A, z, v, cache: dict = None, arch: str = None, repeats: int = 5):
    """Tune the fused pass on A (device, column-major m x n; z, v device n-vectors); returns
    (H, G, ms per pass) and records them in `cache` when given."""
    H, G, ms = binding.fs_tune_pass(ctx, A, z, v, repeats)
    m, n = A.shape
    if cache is not None:
        cache[key(arch or device_arch(), n, m)] = {"H": H, "G": G, "ms": round(ms, 5)}
    return H, G, ms


def apply(ctx, cache: dict, arch: str = None, set_fn=None) -> int:
    """Load the FP64 entries of `arch` into the context; returns how many were loaded."""
    arch = arch or device_arch()
    set_fn = set_fn or binding.fs_set_pass_tuning
    count = 0
    for k, e in sorted(cache.items()):
        a, n, mb, dt = k.split("|")
        if a != arch or dt != "f64":
            continue
        set_fn(ctx, 1 << int(mb), int(n), int(e["H"]), int(e["G"]))
        count += 1
    return count
