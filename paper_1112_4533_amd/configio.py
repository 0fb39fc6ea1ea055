"""Configuration files: the gauge field of a chain plus what is needed to
continue it (paper Sec. 3: configurations are stored for later measurement).

A file is

    8 bytes   magic b"SUNCFG01"
    4 bytes   little-endian uint32: length n of the header
    n bytes   UTF-8 JSON header
    payload   the field as complex128, little-endian, indexed
              [mu][site][i][j] with site = x + L0 (y + L1 (z + L2 t))

The header holds nc, L, the storage the chain ran with, the run parameters
(beta, seed, n_hb, n_or), the chain state (rng_step: the RNG step counter;
sweeps: sweeps done) and the SHA-256 of the payload, which load() checks.
The payload is the library's canonical export, so a chain written from FP32
or two-row storage and read back continues bitwise (every stored value is
exact in FP64).
"""
import hashlib
import json
import os
import struct

import numpy as np

MAGIC = b"SUNCFG01"
REQUIRED = ("nc", "L", "storage", "beta", "seed", "rng_step", "sweeps")


def _payload_shape(nc, L):
    V = 1
    for v in L:
        V *= int(v)
    return (4, V, int(nc), int(nc))


def save(path, field, meta):
    """Writes `field` ((4, V, nc, nc) complex) and the header `meta` (a dict
    with at least the REQUIRED keys) atomically (temporary file + rename)."""
    missing = [k for k in REQUIRED if k not in meta]
    if missing:
        raise ValueError(f"configuration header lacks {missing}")
    shape = _payload_shape(meta["nc"], meta["L"])
    a = np.ascontiguousarray(np.asarray(field, dtype="<c16"))
    if a.shape != shape:
        raise ValueError(f"field shape {a.shape}, header says {shape}")
    payload = a.tobytes()
    head = dict(meta)
    head["L"] = [int(v) for v in meta["L"]]
    head["payload"] = "complex128 little-endian [mu][site][i][j]"
    head["sha256"] = hashlib.sha256(payload).hexdigest()
    hb = json.dumps(head, sort_keys=True).encode("utf-8")
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<I", len(hb)))
        f.write(hb)
        f.write(payload)
    os.replace(tmp, path)


def read_header(path):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a configuration file")
        (n,) = struct.unpack("<I", f.read(4))
        return json.loads(f.read(n).decode("utf-8"))


def load(path):
    """Returns (field as a (4, V, nc, nc) complex128 array, header dict);
    raises ValueError on a bad magic, size or checksum."""
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a configuration file")
        (n,) = struct.unpack("<I", f.read(4))
        head = json.loads(f.read(n).decode("utf-8"))
        payload = f.read()
    shape = _payload_shape(head["nc"], head["L"])
    if len(payload) != 16 * int(np.prod(shape)):
        raise ValueError(f"{path}: payload of {len(payload)} bytes, expected {16 * int(np.prod(shape))}")
    if hashlib.sha256(payload).hexdigest() != head.get("sha256"):
        raise ValueError(f"{path}: checksum mismatch")
    return np.frombuffer(payload, dtype="<c16").reshape(shape).copy(), head


def save_lattice(path, lat, beta, seed, sweeps, **extra):
    """Writes the field and chain state of a sun.Lattice."""
    from . import sun
    field = lat.export().cpu().numpy()
    meta = {"nc": lat.nc, "L": list(lat.L), "storage": sun.DTYPE_NAMES[lat.dtype], "beta": float(beta),
            "seed": int(seed), "rng_step": int(lat.step), "sweeps": int(sweeps)}
    meta.update(extra)
    save(path, field, meta)


def load_lattice(path, storage=None):
    """A sun.Lattice holding the file's field and RNG step counter (in the
    storage it was written from unless `storage` is given), and the header."""
    from . import sun
    import torch
    field, head = load(path)
    lat = sun.Lattice(head["nc"], head["L"], storage or head["storage"])
    lat.import_(torch.from_numpy(field))
    lat.step = int(head["rng_step"])
    return lat, head
