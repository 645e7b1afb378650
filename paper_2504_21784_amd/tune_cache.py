"""On-disk cache of tuned sweep launch shapes.

The launch-shape autotuners time every candidate (waves per band, bands per
workgroup, groups per lane, workgroups per CU) on the live state, which
takes a second or more for a large problem or batch.  The best shape depends
only on the device and on the problem's sweep shape (mesh, groups, angles,
precision, fixup), so it is kept in a JSON file keyed by those and reused:
a later autotune call for the same key applies the stored shape without
timing.

File: ``$SMRT_TUNE_CACHE`` if set, else
``~/.cache/paper_2504_21784_amd/launch_shapes.json``.  Writes go through a
temporary file and an atomic rename, so concurrent writers never leave a
torn file; an unreadable file counts as empty.
"""
import json
import os
import tempfile

DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "paper_2504_21784_amd", "launch_shapes.json")


def problem_key(kind, device, precision, shapes, fixup=0):
    """Cache key of a tuning: kind ("single" or "batch"), the device string,
    the precision (0 FP64, 1 FP32), the fixup flag and, per problem, its
    (nx, ny, G, n_angles), in the batch's order."""
    shp = ";".join(f"{nx}x{ny}g{G}a{na}" for nx, ny, G, na in shapes)
    return f"{kind}|{device}|p{int(precision)}|f{int(fixup)}|{shp}"


class TuneCache:
    def __init__(self, path=None):
        self.path = path or os.environ.get("SMRT_TUNE_CACHE") or DEFAULT_PATH

    def load(self) -> dict:
        try:
            with open(self.path, "r") as f:
                data = json.load(f)
            return data if isinstance(data, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, key):
        """The stored entry {"waves_per_band", "bands_per_group",
        "pairs_per_lane", "workgroups_per_cu", "ms"} or None."""
        e = self.load().get(key)
        need = ("waves_per_band", "bands_per_group", "pairs_per_lane", "workgroups_per_cu", "ms")
        if not isinstance(e, dict) or any(k not in e for k in need):
            return None
        return e

    def put(self, key, entry):
        data = self.load()
        data[key] = dict(entry)
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".launch_shapes.", suffix=".tmp")
        try:
            with os.fdopen(fd, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise
