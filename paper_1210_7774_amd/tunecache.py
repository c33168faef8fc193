"""JSON cache of autotuned launch shapes.

The file maps a key (device, solver form -- precision, smoother, sweeps --,
operator and the systems' sizes) to
the choices mg_tune_get reports: {level size: [block height, tiled]}.  A
missing, unreadable or malformed file or entry is a miss: the caller tunes
again and the entry is rewritten.  Writes go to a temporary file that then
replaces the cache, so a reader never sees half a file.
"""
from __future__ import annotations

import json
import os
import tempfile

VERSION = 1


def key(device: str, form: str, operator: str, sizes) -> str:
    return "v%d|%s|%s|%s|%s" % (VERSION, device, form, operator, ",".join(str(int(n)) for n in sizes))


def _read(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def load(path: str, k: str):
    """Choices stored under k, as {n: (hb, tiled)}, or None on any miss."""
    ent = _read(path).get(k)
    if not isinstance(ent, dict) or not ent:
        return None
    out = {}
    try:
        for n, v in ent.items():
            hb, tiled = v
            n, hb = int(n), int(hb)
            if n < 1 or not 2 <= hb <= 256 or not isinstance(tiled, bool):
                return None
            out[n] = (hb, tiled)
    except (TypeError, ValueError):
        return None
    return out


def store(path: str, k: str, choices) -> None:
    data = _read(path)
    data[k] = {str(int(n)): [int(hb), bool(t)] for n, (hb, t) in sorted(choices.items())}
    d = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(prefix=".tune", dir=d)
    try:
        with os.fdopen(fd, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise
