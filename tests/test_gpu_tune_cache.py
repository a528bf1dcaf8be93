"""The batched CG's launch-shape cache file (PGCP_TUNE_CACHE).

Tuning a batch appends its shape to the file; a file line for a batch, with
this GPU's and this build's tag, replaces the tuning (no probe launches) and
its shape is the one launched; a line with another tag is ignored.  All in this
process: a second process cannot make cooperative launches on the GPU while
this one holds it.  The library also keeps shapes in memory for the process,
so each part uses a mesh of its own and the file is read once per path."""
import sys

import pytest

from synth import small_grid_case

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-tune-cache]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_1903_12359_amd as pg
    pg.load_library()
    assert torch.cuda.is_available()
    c = pg.Context(0)
    yield c
    c.close()


def _key(row0):
    """The batch key of an FP64 DNCP solve: precision 0, coupled system, the
    piece count and every piece's 64-row slices."""
    k = len(row0) - 1
    return "0:1:%d" % k + "".join(",%d" % ((row0[i + 1] - row0[i]) // 64) for i in range(k))


def _plan_key(ctx, case):
    import paper_1903_12359_amd as pg
    plan = pg.Plan(ctx, case.V, case.F, case.label, "free")
    row0 = plan.rows()
    plan.close()
    return _key(row0)


def _dncp(ctx, case, cache, monkeypatch, capfd):
    """FP64 DNCP solve of `case` with the cache file `cache`; returns the
    report, the tuning lines the library printed and the batch's key."""
    import torch
    import paper_1903_12359_amd as pg
    for k in ("PGCP_PCG_CFG", "PGCP_PCG_CFG64", "PGCP_PCG_CFG32", "PGCP_TUNE"):
        monkeypatch.delenv(k, raising=False)
    monkeypatch.setenv("PGCP_TUNE_CACHE", str(cache))
    monkeypatch.setenv("PGCP_VERBOSE", "1")
    capfd.readouterr()
    plan = pg.Plan(ctx, case.V, case.F, case.label, "free")
    pg.assemble_cotan(ctx, plan, torch.from_numpy(case.V).to("cuda:0"))
    _, rep = pg.local_param(ctx, plan, precision="fp64", tol=1e-10)
    row0 = plan.rows()
    plan.close()
    monkeypatch.delenv("PGCP_VERBOSE")
    err = capfd.readouterr().err
    tunes = [ln for ln in err.splitlines() if ln.startswith("[pgcp] tune ")]
    key = _key(row0)
    say(case.name, "tuning lines", len(tunes), "shape", rep.cg_block, rep.rows_per_thread, rep.cg_stream)
    assert (rep.status == 0).all()
    return rep, tunes, key


def test_tune_cache_file(ctx, tmp_path, monkeypatch, capfd):
    # tuning appends the batch's line, tagged with the GPU and the build
    rep, tunes, key = _dncp(ctx, small_grid_case(65, 3, 2, seed=7), tmp_path / "a.txt", monkeypatch, capfd)
    assert tunes
    lines = [ln.split() for ln in (tmp_path / "a.txt").read_text().splitlines()]
    assert [ln[1] for ln in lines] == [key]
    tag = lines[0][0]
    assert tag.startswith("gfx950") and len(lines[0]) == 5
    assert (int(lines[0][2]), int(lines[0][4])) == (rep.cg_block, rep.cg_stream)

    # a line with this tag is used: no probes, its shape is launched
    case = small_grid_case(61, 2, 3, seed=11)
    key_b = _plan_key(ctx, case)
    (tmp_path / "b.txt").write_text("%s %s 512 1 1\n" % (tag, key_b))
    rep, tunes, key = _dncp(ctx, case, tmp_path / "b.txt", monkeypatch, capfd)
    assert key == key_b and tunes == []
    assert (rep.cg_block, rep.cg_stream) == (512, 1)
    assert (tmp_path / "b.txt").read_text().splitlines() == ["%s %s 512 1 1" % (tag, key_b)]

    # a line of another build is ignored: the batch is tuned and its line appended
    case = small_grid_case(53, 3, 3, seed=13)
    key_c = _plan_key(ctx, case)
    other = "gfx950:other/256/Jan_1_2000/00:00:00"
    (tmp_path / "c.txt").write_text("%s %s 512 1 1\n" % (other, key_c))
    rep, tunes, key = _dncp(ctx, case, tmp_path / "c.txt", monkeypatch, capfd)
    assert key == key_c and tunes
    lines = (tmp_path / "c.txt").read_text().splitlines()
    assert len(lines) == 2 and lines[1].split()[:2] == [tag, key_c]
