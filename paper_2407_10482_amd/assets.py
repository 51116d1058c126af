"""Scene assets on disk: the checkpoint of a baked scene.

A trained scene is frozen into the arrays the render path reads: the
multi-resolution hash tables, the baked model's coarse features and
attention parameters (F~ and A, Sec. 4.1-4.2), the occupancy grid O or the
fine grid its pyramid is built from, with the distance grid G (Sec. 4.3),
the deferred MLP (Eq. 5) and, optionally, the proposal network's weights.
Here such a scene is a directory of one ``.npy`` file per array beside
``manifest.json``, which holds the renderer descriptor (the arguments of
``Renderer``) and, per file, its SHA-256 (of the whole ``.npy`` file, so
``sha256sum`` reproduces it), shape and dtype.

Reading checks the manifest's format, every listed file's hash, and each
array's dtype and shape against both the manifest and the descriptor
before it returns anything; ``.npy`` files are read with
``allow_pickle=False`` and the manifest as JSON, so nothing in the
directory is executed.  Any mismatch raises ``AssetError`` naming the
file.  Host code only (numpy): ``Renderer.from_assets`` moves the arrays to
the device and loads them through the C ABI.
"""
from __future__ import annotations

import hashlib
import io
import json
import os
from typing import Dict, Mapping, Optional, Tuple

import numpy as np

from ._lib import MODEL_BAKED, coarse_channels, mlp_param_count

FORMAT = "ngprt-scene-assets/1"
MANIFEST = "manifest.json"
PROPOSAL_PARAMS = 7556

# name -> numpy dtype of the file; the loader each feeds is fixed by the name
DTYPES = {
    "tables": np.float32,         # [L][T][9]: 8 features + density logit per entry
    "occ": np.uint8,              # [R][R][R] occupancy O (single-level march)
    "dist": np.uint8,             # [R][R][R] distance grid G (optional; else built from occ)
    "occ_fine": np.uint8,         # [F][F][F] finest occupancy of the pyramid
    "mlp": np.float32,            # deferred MLP parameters
    "coarse_index": np.int32,     # [nb][nb][nb] atlas row of each 8^3 block or -1
    "coarse_atlas": np.float32,   # [n_blocks][8][8][8][C]
    "coarse_default": np.float32, # [C] value of every vertex of an empty block
    "proposal": np.float32,       # [7556] proposal network master weights
}

# descriptor keys: the arguments of Renderer, in JSON types
DESCRIPTOR_KEYS = ("resolutions", "log2_table_size", "table_dtype", "domain", "roi_half", "occ_res",
                   "step", "max_samples", "t_threshold", "feature_model", "coarse_res", "occ_levels",
                   "occ_fine_res", "use_distance", "mlp_dims", "aggregation", "gate_params")


class AssetError(ValueError):
    """A scene directory that does not match its manifest or descriptor."""


def _sha256(path: str) -> str:
    h = hashlib.sha256()
    with open(path, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 22), b""):
            h.update(chunk)
    return h.hexdigest()


def normalise_descriptor(desc: Mapping) -> Dict:
    """The descriptor with every key present and in plain JSON types."""
    missing = [k for k in DESCRIPTOR_KEYS if k not in desc]
    if missing:
        raise AssetError(f"descriptor lacks {missing}")
    extra = [k for k in desc if k not in DESCRIPTOR_KEYS]
    if extra:
        raise AssetError(f"descriptor has unknown keys {extra}")
    d = {}
    for k in DESCRIPTOR_KEYS:
        v = desc[k]
        if k in ("resolutions", "mlp_dims"):
            d[k] = [int(x) for x in v]
        elif k == "gate_params":
            d[k] = [float(x) for x in v]
        elif k in ("roi_half", "step", "t_threshold"):
            d[k] = float(v)
        elif k == "use_distance":
            d[k] = bool(v)
        else:
            d[k] = int(v)
    if len(d["mlp_dims"]) != 4:
        raise AssetError("descriptor mlp_dims must be (in, hidden, hidden, out)")
    return d


def expected_shape(desc: Mapping, name: str, arrays: Mapping[str, np.ndarray]) -> Optional[Tuple[int, ...]]:
    """Shape the descriptor fixes for an asset (None for the atlas's block
    count, which only has to agree with the index)."""
    L = len(desc["resolutions"])
    R, F = desc["occ_res"], desc["occ_fine_res"]
    C = coarse_channels(L, desc["aggregation"])
    if name == "tables":
        return (L, 1 << desc["log2_table_size"], 9)
    if name in ("occ", "dist"):
        return (R, R, R)
    if name == "occ_fine":
        return (F, F, F)
    if name == "mlp":
        return (mlp_param_count(desc["mlp_dims"]),)
    if name == "coarse_index":
        nb = (desc["coarse_res"] + 1 + 7) // 8
        return (nb, nb, nb)
    if name == "coarse_atlas":
        return None
    if name == "coarse_default":
        return (C,)
    if name == "proposal":
        return (PROPOSAL_PARAMS,)
    raise AssetError(f"unknown asset {name!r}")


def required_assets(desc: Mapping) -> Tuple[str, ...]:
    req = ["tables", "mlp", "occ_fine" if desc["occ_levels"] else "occ"]
    if desc["feature_model"] == MODEL_BAKED:
        req += ["coarse_index", "coarse_atlas", "coarse_default"]
    return tuple(req)


def check_assets(desc: Mapping, arrays: Mapping[str, np.ndarray]) -> None:
    """Raise AssetError unless the arrays are the scene the descriptor describes."""
    for name in arrays:
        if name not in DTYPES:
            raise AssetError(f"unknown asset {name!r} (known: {sorted(DTYPES)})")
    for name in required_assets(desc):
        if name not in arrays:
            raise AssetError(f"asset {name!r} is required by this descriptor")
    if "dist" in arrays and desc["occ_levels"]:
        raise AssetError("a pyramid scene builds its distance grid from occ_fine: drop 'dist'")
    if "occ" in arrays and desc["occ_levels"]:
        raise AssetError("a pyramid scene takes 'occ_fine', not 'occ'")
    if "occ_fine" in arrays and not desc["occ_levels"]:
        raise AssetError("'occ_fine' needs occ_levels > 0 in the descriptor")
    for name, a in arrays.items():
        if a.dtype != np.dtype(DTYPES[name]):
            raise AssetError(f"asset {name!r} must be {np.dtype(DTYPES[name])}, got {a.dtype}")
        shape = expected_shape(desc, name, arrays)
        if shape is not None and tuple(a.shape) != shape:
            raise AssetError(f"asset {name!r} must have shape {shape}, got {tuple(a.shape)}")
    if desc["feature_model"] == MODEL_BAKED:
        C = coarse_channels(len(desc["resolutions"]), desc["aggregation"])
        atlas, index = arrays["coarse_atlas"], arrays["coarse_index"]
        if atlas.ndim != 5 or tuple(atlas.shape[1:]) != (8, 8, 8, C):
            raise AssetError(f"asset 'coarse_atlas' must have shape (n_blocks, 8, 8, 8, {C}), "
                             f"got {tuple(atlas.shape)}")
        n_blocks = atlas.shape[0]
        if index.size and (index.min() < -1 or index.max() >= n_blocks):
            raise AssetError(f"asset 'coarse_index' holds rows outside -1..{n_blocks - 1}")


def save_scene(path: str, descriptor: Mapping, arrays: Mapping[str, np.ndarray]) -> Dict:
    """Write the arrays and the manifest into directory ``path`` (created if
    needed; existing asset files of the same names are replaced).  Arrays
    must already have the asset dtypes: nothing is converted.  The manifest
    is written last, through a temporary file, so a directory with a
    manifest holds every file it lists.  Returns the manifest."""
    desc = normalise_descriptor(descriptor)
    arrays = {k: np.ascontiguousarray(np.asarray(v)) for k, v in arrays.items()}
    check_assets(desc, arrays)
    os.makedirs(path, exist_ok=True)
    files = {}
    for name in sorted(arrays):
        fname = name + ".npy"
        fpath = os.path.join(path, fname)
        np.save(fpath, arrays[name], allow_pickle=False)
        files[name] = {"file": fname, "sha256": _sha256(fpath), "dtype": str(arrays[name].dtype),
                       "shape": list(arrays[name].shape)}
    manifest = {"format": FORMAT, "descriptor": desc, "assets": files}
    tmp = os.path.join(path, MANIFEST + ".tmp")
    with open(tmp, "w") as f:
        json.dump(manifest, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, os.path.join(path, MANIFEST))
    return manifest


def read_manifest(path: str) -> Dict:
    mpath = os.path.join(path, MANIFEST)
    if not os.path.isfile(mpath):
        raise AssetError(f"no {MANIFEST} in {path}")
    try:
        with open(mpath) as f:
            manifest = json.load(f)
    except (OSError, ValueError) as e:
        raise AssetError(f"{mpath}: unreadable manifest ({e})") from None
    if not isinstance(manifest, dict) or manifest.get("format") != FORMAT:
        raise AssetError(f"{mpath}: format is not {FORMAT!r}")
    if not isinstance(manifest.get("assets"), dict) or not isinstance(manifest.get("descriptor"), dict):
        raise AssetError(f"{mpath}: needs 'descriptor' and 'assets' objects")
    return manifest


def read_scene(path: str) -> Tuple[Dict, Dict[str, np.ndarray]]:
    """The descriptor and arrays of a scene directory, every file verified
    against the manifest and the descriptor first."""
    manifest = read_manifest(path)
    desc = normalise_descriptor(manifest["descriptor"])
    arrays = {}
    for name, entry in sorted(manifest["assets"].items()):
        if name not in DTYPES:
            raise AssetError(f"manifest lists unknown asset {name!r}")
        if not isinstance(entry, dict):
            raise AssetError(f"asset {name!r}: manifest entry must be an object")
        fname = entry.get("file", "")
        if not isinstance(fname, str):
            raise AssetError(f"asset {name!r}: manifest 'file' must be a string")
        if os.path.basename(fname) != fname or not fname.endswith(".npy"):
            raise AssetError(f"asset {name!r}: file {fname!r} must be a .npy file in the scene directory")
        fpath = os.path.join(path, fname)
        if not os.path.isfile(fpath):
            raise AssetError(f"asset {name!r}: {fname} is missing")
        # the bytes that are hashed are the bytes that are parsed
        with open(fpath, "rb") as f:
            data = f.read()
        digest = hashlib.sha256(data).hexdigest()
        if digest != entry.get("sha256"):
            raise AssetError(f"asset {name!r}: {fname} has SHA-256 {digest}, the manifest says "
                             f"{entry.get('sha256')}")
        try:
            a = np.load(io.BytesIO(data), allow_pickle=False)
        except ValueError as e:
            raise AssetError(f"asset {name!r}: {fname} is not a plain array file ({e})") from None
        if str(a.dtype) != entry.get("dtype") or list(a.shape) != entry.get("shape"):
            raise AssetError(f"asset {name!r}: {fname} holds {a.dtype} {list(a.shape)}, the manifest says "
                             f"{entry.get('dtype')} {entry.get('shape')}")
        arrays[name] = a
    check_assets(desc, arrays)
    return desc, arrays
