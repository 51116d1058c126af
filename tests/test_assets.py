"""Scene asset directories (host side): round trip, hash verification and
refusal of files that do not match their manifest or descriptor."""
import hashlib
import json
import os

import numpy as np
import pytest

from helpers import renderer_kwargs, scene_assets
from paper_2407_10482_amd import assets
from paper_2407_10482_amd.assets import AssetError


def _save(tmp_path, name="tiny", **kw):
    desc = renderer_kwargs(name)
    arrays = scene_assets(name, **kw)
    path = str(tmp_path / name)
    manifest = assets.save_scene(path, desc, arrays)
    return path, desc, arrays, manifest


@pytest.mark.parametrize("name", ["tiny", "baked_tiny_pyramid", "tiny_view", "baked_tiny_shared_v"])
def test_round_trip_is_bit_exact(tmp_path, name):
    path, desc, arrays, manifest = _save(tmp_path, name, with_dist=True)
    rdesc, rarrays = assets.read_scene(path)
    assert rdesc == assets.normalise_descriptor(desc)
    assert sorted(rarrays) == sorted(arrays)
    for k, a in arrays.items():
        assert rarrays[k].dtype == a.dtype and rarrays[k].shape == a.shape
        assert np.array_equal(rarrays[k].view(np.uint8), np.ascontiguousarray(a).view(np.uint8)), k
    # the recorded digests are those of the whole files
    for k, e in manifest["assets"].items():
        with open(os.path.join(path, e["file"]), "rb") as f:
            assert hashlib.sha256(f.read()).hexdigest() == e["sha256"]
    with open(os.path.join(path, assets.MANIFEST)) as f:
        assert json.load(f) == manifest


def test_mlp_param_counts():
    from paper_2407_10482_amd._lib import mlp_param_count
    assert mlp_param_count((7, 16, 16, 3)) == 451
    assert mlp_param_count((23, 64, 64, 3)) == 5891


def test_changed_byte_is_refused(tmp_path):
    path, *_ = _save(tmp_path)
    fpath = os.path.join(path, "tables.npy")
    with open(fpath, "r+b") as f:
        f.seek(os.path.getsize(fpath) // 2)
        b = f.read(1)
        f.seek(-1, 1)
        f.write(bytes([b[0] ^ 1]))
    with pytest.raises(AssetError, match="'tables'.*SHA-256"):
        assets.read_scene(path)


def test_missing_and_truncated_files_are_refused(tmp_path):
    path, *_ = _save(tmp_path)
    fpath = os.path.join(path, "mlp.npy")
    with open(fpath, "rb") as f:
        data = f.read()
    with open(fpath, "wb") as f:
        f.write(data[:-4])
    with pytest.raises(AssetError, match="'mlp'"):
        assets.read_scene(path)
    os.remove(fpath)
    with pytest.raises(AssetError, match="missing"):
        assets.read_scene(path)
    os.remove(os.path.join(path, assets.MANIFEST))
    with pytest.raises(AssetError, match="no manifest.json"):
        assets.read_scene(path)


def _rewrite_manifest(path, edit):
    mpath = os.path.join(path, assets.MANIFEST)
    with open(mpath) as f:
        m = json.load(f)
    edit(m)
    with open(mpath, "w") as f:
        json.dump(m, f)


def test_manifest_format_and_paths_are_checked(tmp_path):
    path, *_ = _save(tmp_path)
    _rewrite_manifest(path, lambda m: m.update(format="something-else/9"))
    with pytest.raises(AssetError, match="format"):
        assets.read_scene(path)
    path, *_ = _save(tmp_path / "b")
    _rewrite_manifest(path, lambda m: m["assets"]["mlp"].update(file="../mlp.npy"))
    with pytest.raises(AssetError, match="in the scene directory"):
        assets.read_scene(path)
    path, *_ = _save(tmp_path / "c")
    _rewrite_manifest(path, lambda m: m["assets"].update(extra=dict(m["assets"]["mlp"])))
    with pytest.raises(AssetError, match="unknown asset 'extra'"):
        assets.read_scene(path)
    path, *_ = _save(tmp_path / "d")
    _rewrite_manifest(path, lambda m: m["assets"]["mlp"].update(shape=[452]))
    with pytest.raises(AssetError, match="the manifest says"):
        assets.read_scene(path)
    path, *_ = _save(tmp_path / "e")
    _rewrite_manifest(path, lambda m: m["assets"].update(mlp=["mlp.npy"]))
    with pytest.raises(AssetError, match="must be an object"):
        assets.read_scene(path)


def test_object_array_is_not_unpickled(tmp_path):
    """A file that needs unpickling is refused even when its digest matches."""
    path, *_ = _save(tmp_path)
    fpath = os.path.join(path, "mlp.npy")
    np.save(fpath, np.array([{"a": 1}, None], dtype=object), allow_pickle=True)
    with open(fpath, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    _rewrite_manifest(path, lambda m: m["assets"]["mlp"].update(sha256=digest))
    with pytest.raises(AssetError, match="not a plain array file"):
        assets.read_scene(path)


def test_save_refuses_arrays_the_descriptor_does_not_describe(tmp_path):
    desc = renderer_kwargs("tiny")
    good = scene_assets("tiny")
    cases = [
        (dict(good, tables=good["tables"].astype(np.float64)), "must be float32"),
        (dict(good, tables=good["tables"][:, :100]), "must have shape"),
        (dict(good, foo=good["mlp"]), "unknown asset 'foo'"),
        ({k: v for k, v in good.items() if k != "mlp"}, "'mlp' is required"),
        (dict(good, occ_fine=np.zeros((4, 4, 4), np.uint8)), "occ_levels"),
    ]
    for arrays, msg in cases:
        with pytest.raises(AssetError, match=msg):
            assets.save_scene(str(tmp_path / "x"), desc, arrays)
    pdesc = renderer_kwargs("baked_tiny_pyramid")
    pgood = scene_assets("baked_tiny_pyramid")
    with pytest.raises(AssetError, match="takes 'occ_fine'"):
        assets.save_scene(str(tmp_path / "y"), pdesc, dict(pgood, occ=np.zeros((64,) * 3, np.uint8)))
    bad_index = pgood["coarse_index"].copy()
    bad_index.flat[0] = pgood["coarse_atlas"].shape[0]
    with pytest.raises(AssetError, match="rows outside"):
        assets.save_scene(str(tmp_path / "z"), pdesc, dict(pgood, coarse_index=bad_index))
    with pytest.raises(AssetError, match="coarse_atlas"):
        assets.save_scene(str(tmp_path / "w"), pdesc, dict(pgood, coarse_atlas=pgood["coarse_atlas"][..., :8]))
    with pytest.raises(AssetError, match="descriptor lacks"):
        assets.save_scene(str(tmp_path / "v"), {k: v for k, v in desc.items() if k != "step"}, good)
