"""The ray-bundle shape tuner's host logic, with a fake device timer: the
per-class choice, the batched coordinate descent (each class ends on its own
fastest shape, with every grid of the class set to it), and the table file."""
from types import SimpleNamespace

from paper_2112_13169_amd import autotune


class FakeVg:
    VG_SPINNING = 1

    def __init__(self, sizes):
        self.sizes = sizes          # vox_size -> (vd, hw, hh, rays)

    def vg_fan_sizes(self, sensor, vox_size):
        return self.sizes[vox_size]


def test_fan_class_buckets_depth_and_aspect():
    lib = FakeVg({0.05: (160, 160, 92, 0), 0.051: (157, 157, 90, 0), 0.1: (80, 80, 46, 0)})
    pin = SimpleNamespace(kind=0)
    spin = SimpleNamespace(kind=1)
    # nearby voxel sizes share a class; halving the depth moves two sqrt(2) buckets
    assert autotune.fan_class(pin, 0.05, lib) == autotune.fan_class(pin, 0.051, lib)
    a, b = autotune.fan_class(pin, 0.05, lib), autotune.fan_class(pin, 0.1, lib)
    assert a[1] == b[1] and a[2] - b[2] == 2
    # a spinning sensor has no aspect
    assert autotune.fan_class(spin, 0.05, lib)[1] == 0 and autotune.fan_class(spin, 0.05, lib)[0] == 1


def test_tune_batch_finds_each_class_optimum():
    target = {"a": 5, "b": 1, "c": 3}
    owner = {1: "a", 2: "a", 3: "a", 4: "b", 5: "c", 6: "c"}
    tile = {}
    calls = []

    def set_tile(h, w):
        tile[h] = w

    def time_rays():
        # separable cost: each grid pays for its distance from its class optimum
        calls.append(dict(tile))
        return 1.0 + sum((tile[h] - target[owner[h]]) ** 2 for h in owner)

    classes = {"b": [4], "a": [1, 2, 3], "c": [5, 6]}
    table = autotune.tune_batch(classes, set_tile, time_rays, reps=2)
    assert {c: b for c, (b, _) in table.items()} == target
    assert all(tile[h] == target[owner[h]] for h in owner)
    assert list(table) == ["a", "c", "b"]                  # largest class first
    assert set(table["a"][1]) == set(autotune.SHAPES)
    # every timing of a shape is one warm run plus `reps` timed runs
    assert len(calls) == len(classes) * len(autotune.SHAPES) * 3


def test_table_round_trip_and_default(tmp_path):
    lib = FakeVg({0.05: (160, 160, 92, 0), 0.2: (40, 40, 23, 0)})
    pin = SimpleNamespace(kind=0)
    table = {autotune.fan_class(pin, 0.05, lib): (2, {w: 1.0 + w for w in autotune.SHAPES})}
    path = tmp_path / "tiles.json"
    autotune.save(table, str(path))
    back = autotune.load(str(path))
    assert back == table
    assert autotune.choose(back, pin, 0.05, lib) == 2
    assert autotune.choose(back, pin, 0.2, lib) == 3            # untuned class: 8 x 8
