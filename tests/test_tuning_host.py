"""Host side of the launch tuning (no GPU needed): vs_set_tuning validates and round-trips, NULL
restores the defaults, a rejected setting changes nothing; the autotuner's classes, cache keys and
JSON cache."""
import pytest

from paper_1701_03572_amd import tuning as T
from paper_1701_03572_amd import vstab as V


@pytest.fixture(autouse=True)
def defaults():
    T.set_tuning(None)
    yield
    T.set_tuning(None)


def test_defaults_and_round_trip():
    assert T.get_tuning() == T.Tuning(8, 8, 8, 1)
    t = T.Tuning(1, 65536, 3, 4)
    T.set_tuning(t)
    assert T.get_tuning() == t
    T.set_tuning(T.Tuning(0, 0, 0, 0, 0, 0))    # zeros select the defaults
    assert T.get_tuning() == T.Tuning(8, 8, 8, 1, 0, 2048)
    t = T.Tuning(det_rows=30, fit_groups=512)
    T.set_tuning(t)
    assert T.get_tuning() == t


@pytest.mark.parametrize("bad", [T.Tuning(-1, 8, 8, 1), T.Tuning(8, 65537, 8, 1), T.Tuning(8, 8, 8, 3),
                                 T.Tuning(8, 8, 8, 8), T.Tuning(det_rows=11), T.Tuning(det_rows=241),
                                 T.Tuning(fit_groups=63), T.Tuning(fit_groups=16385)])
def test_rejected_settings_change_nothing(bad):
    T.set_tuning(T.Tuning(1, 1, 1, 2))
    with pytest.raises(V.VsError):
        T.set_tuning(bad)
    assert T.get_tuning() == T.Tuning(1, 1, 1, 2)


def test_classes_and_keys():
    assert T.resolution_class(320, 240) == "320x240"
    assert T.resolution_class(321, 240) == "640x480"
    assert T.resolution_class(1920, 1080) == "1920x1080"
    assert T.resolution_class(4096, 2160) == ">3840x2160"
    assert T.k_class(50) == "K<=256" and T.k_class(1000) == "K<=1024" and T.k_class(5000) == "K>4096"
    assert T.cache_key("gfx950", 1920, 1080, 1000) == "gfx950/1920x1080/K<=1024"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert T.lookup("gfx950", 640, 480, 500, path) is None
    t = T.Tuning(1, 8, 65536, 2)
    T.store(T.cache_key("gfx950", 640, 480, 500), t, {"lk": {"8/1": 1.0}}, {"frames": 21}, path)
    T.store(T.cache_key("gfx950", 1920, 1080, 1000), T.Tuning(), {}, {}, path)
    assert T.lookup("gfx950", 600, 400, 300, path) == t           # same classes
    assert T.lookup("gfx942", 640, 480, 500, path) is None        # another architecture
    assert T.load_cache(path)["gfx950/640x480/K<=1024"]["timings_ms"]["lk"]["8/1"] == 1.0
