"""Host logic of the autotuner: the cache key and the JSON cache (no GPU)."""
import json
import types

from paper_2105_01612_amd import autotune as at


def fake_plan(nx=64, ny=64, nz=64, batch=1, prec="fp32", op="ddo"):
    return types.SimpleNamespace(nx=nx, ny=ny, nz=nz, batch=batch, prec=prec, op=op)


def test_cache_key_names_every_field_that_changes_the_tuning():
    base = at.cache_key(fake_plan(), arch="gfx950")
    assert base == "gfx950|64x64x64|b1|fp32|ddo"
    variants = [fake_plan(nx=128), fake_plan(ny=32), fake_plan(nz=96), fake_plan(batch=64), fake_plan(prec="fp64"),
                fake_plan(op="cdo")]
    keys = {at.cache_key(p, arch="gfx950") for p in variants}
    assert base not in keys and len(keys) == len(variants)
    assert at.cache_key(fake_plan(), arch="gfx942") != base


def test_cache_json_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv(at.CACHE_ENV, str(path))
    assert at.cache_path() == str(path)
    assert at.load_cache() == {}                      # absent file: empty cache
    entry = {"tune": {"tx_y": 32, "tx_z": 64, "rw_x": 4, "chunk": 0, "radix16": 6, "schedule": 5, "tc_zp": 0,
                      "radix4": 0, "xsplit": 2},
             "resolved": {"tx_y": 32, "tx_z": 64, "rw_x": 4, "chunk": 129, "radix16": 6, "schedule": 5,
                          "tc_zp": 0, "radix4": 0, "xsplit": 2},
             "pass_ms": {"z_r2c": 0.147, "x_proj": 0.18}, "project_ms": 0.94}
    key = at.cache_key(fake_plan(256, 256, 256), arch="gfx950")
    at.save_cache({key: entry})
    assert path.exists() and not (tmp_path / "sub" / "tune.json.tmp").exists()
    assert at.load_cache() == {key: entry}
    assert json.loads(path.read_text())[key]["tune"]["radix16"] == 6


def test_corrupt_cache_reads_as_empty(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    monkeypatch.setenv(at.CACHE_ENV, str(path))
    assert at.load_cache() == {}


def test_cached_entry_is_applied_without_trials(tmp_path, monkeypatch):
    """A cache hit applies the stored tuning once and launches nothing else."""
    monkeypatch.setenv(at.CACHE_ENV, str(tmp_path / "tune.json"))
    plan = fake_plan()
    calls = []
    plan.tune = lambda **kw: calls.append(("tune", kw))
    plan.project = lambda *a, **k: calls.append(("project",))
    key = at.cache_key(plan, arch="gfx950")
    monkeypatch.setattr(at, "_arch", lambda: "gfx950")
    at.save_cache({key: {"tune": {"tx_y": 16, "schedule": 3}, "resolved": {}, "pass_ms": {}, "project_ms": 0.0}})
    got = at.autotune(plan, None, None, use_cache=True)
    assert got["tune"] == {"tx_y": 16, "schedule": 3}
    assert calls == [("tune", {"tx_y": 16, "schedule": 3})]


def test_apply_cached_reads_the_named_file_and_never_searches(tmp_path, monkeypatch):
    """apply_cached (serving slots): the entry of the plan's configuration in the named file is
    applied; a configuration without one keeps its defaults, and nothing is timed or written."""
    monkeypatch.setenv(at.CACHE_ENV, str(tmp_path / "default.json"))      # not the file named below
    monkeypatch.setattr(at, "_arch", lambda: "gfx950")
    path = tmp_path / "classes.json"
    path.write_text(json.dumps({"gfx950|128x128x128|b1|fp32|ddo": {"tune": {"tc_zp": 8, "zp_e": 4}}}))
    calls = []

    def mk(n):
        p = fake_plan(n, n, n)
        p.tune = lambda **kw: calls.append((n, kw))
        p.project = lambda *a, **k: calls.append((n, "project"))
        return p

    assert at.apply_cached(mk(128), str(path)) == {"tc_zp": 8, "zp_e": 4}
    assert at.apply_cached(mk(64), str(path)) is None
    assert at.apply_cached(mk(128), str(tmp_path / "absent.json")) is None
    assert calls == [(128, {"tc_zp": 8, "zp_e": 4})]
    assert not (tmp_path / "default.json").exists()
