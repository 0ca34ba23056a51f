"""The C-ABI library loads on a machine without a GPU and exports every symbol
that include/poolboil.h declares; host-only helpers work there."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from helpers import derived
from paper_1911_10747_amd import workloads as W

HEADER = os.path.join(ROOT, "include", "poolboil.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1911_10747_amd import poolboil as pb
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(pb.lib, n), n
    assert sorted(pb.EXPORTED) == names
    assert pb.lib.pb_version() == 1


def test_config_struct_matches_header_field_order():
    from paper_1911_10747_amd import poolboil as pb
    src = open(HEADER).read()
    body = src[src.index("typedef struct pb_config"):src.index("} pb_config;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in re.findall(r"(?:int32_t|uint32_t|double)\s+([^;]+);", body):
        fields += [f.strip() for f in decl.split(",")]
    assert fields == [f for f, _ in pb.Config._fields_]


def test_host_eos_helpers_match_oracle():
    """The library's own Tc formula and Newton-based Maxwell construction agree
    with the oracle's independent bisection construction."""
    from paper_1911_10747_amd import poolboil as pb
    P = W.BASE_PARAMS
    for a in (2 / 49, 3 / 49):
        d = derived(a, P["b"], P["R"], P["omega"])
        Tc = pb.critical_temperature(a, P["b"], P["R"])
        assert Tc == pytest.approx(d["Tc"], rel=1e-14)
        rl, rv = pb.coexistence(a, P["b"], P["R"], P["omega"], Tc, 0.86 * Tc)
        assert rl == pytest.approx(d["rho_L"], rel=1e-10)
        assert rv == pytest.approx(d["rho_V"], rel=1e-10)
        from oracle import eos
        h = pb.latent_heat(a, P["b"], P["R"], P["omega"], Tc, 0.86 * Tc)
        assert h == pytest.approx(eos.latent_heat(0.86 * d["Tc"], a, P["b"], P["R"], P["omega"], d["Tc"]), rel=1e-6)
        psi = pb.eos_psi(a, P["b"], P["R"], P["omega"], Tc, -1.0, rl, 0.86 * Tc)
        assert psi == pytest.approx(d["psi_L"], rel=1e-10)


def test_invalid_configs_rejected_without_gpu():
    """Validation happens on the host before any device call."""
    from paper_1911_10747_amd import poolboil as pb
    P = dict(W.BASE_PARAMS, Tc=0.07, rho_L=6.5, rho_V=0.38, rho_S=19.5)
    base = dict(nx=8, ny_fluid=8, ny_solid=4, **P)
    for bad in (dict(nx=0), dict(ny_solid=0), dict(precision=7), dict(flags=0x100), dict(G=1.0),
                dict(tile_x=48, tile_y=3), dict(thermal_tile=99), dict(rho_V=7.0), dict(s_e=2.5)):
        cfg = pb.make_config(**dict(base, **bad))
        with pytest.raises(pb.PbError) as ei:
            pb.domain_bytes(cfg)
        assert ei.value.code == pb.PB_EINVAL
    assert pb.domain_bytes(pb.make_config(**base)) > 0
    # 32-bit element offsets: nine population planes of 14600 x 32768 nodes
    # pass 2^32 (about 50 GB in FP32, so the memory itself would fit)
    big = pb.make_config(**dict(base, nx=32768, ny_fluid=14600, ny_solid=64))
    with pytest.raises(pb.PbError) as ei:
        pb.domain_bytes(big)
    assert ei.value.code == pb.PB_EINVAL and "32-bit" in str(ei.value)
    assert pb.domain_bytes(pb.make_config(**dict(base, nx=32768, ny_fluid=14500, ny_solid=64))) > 0


def test_energy_strip_height_by_domain_size():
    """thermal_tile 0 picks the energy strips from the domain size: the
    tallest strips of which there are enough to give every SIMD slot one (the
    4096x2048 + 4096x64 roofline domain: 74 x 59 = 4366 strips of 36 rows with
    FP32-deviation storage; FP64 strips stop at 28 rows, 74 x 76 = 5624),
    8-row strips for a small domain (400x400 + 400x20: 8 x 53 = 424 strips),
    and 1..7 select 28, 20, 24, 16, 12, 8 or 36 rows explicitly.  Host only."""
    from paper_1911_10747_amd import poolboil as pb
    P = dict(W.BASE_PARAMS, Tc=0.07, rho_L=6.5, rho_V=0.38, rho_S=19.5)
    rows = lambda **kw: pb.thermal_strip_rows(pb.make_config(**dict(P, **kw)))
    assert rows(nx=4096, ny_fluid=2048, ny_solid=64, precision=1) == 36
    assert rows(nx=4096, ny_fluid=2048, ny_solid=64, precision=0) == 28
    assert rows(nx=400, ny_fluid=400, ny_solid=20) == 8
    assert rows(nx=2048, ny_fluid=1024, ny_solid=51) == 12    # 37 x 90 = 3330 strips of 12 rows
    assert [rows(nx=400, ny_fluid=400, ny_solid=20, thermal_tile=v) for v in range(1, 8)] == [28, 20, 24, 16, 12, 8, 36]
    with pytest.raises(pb.PbError):
        rows(nx=400, ny_fluid=400, ny_solid=20, thermal_tile=8)


def _cover(strips, doms, ncol=56):
    """Every (column block, thermal row) of every domain covered exactly once."""
    for j, (nx, nr) in enumerate(doms):
        grid = np.zeros((nr, (nx + ncol - 1) // ncol), dtype=np.int32)
        for d, x0, y0, rows in strips:
            if d == j:
                assert x0 % ncol == 0 and 0 <= x0 < nx and 0 <= y0 < nr
                grid[y0:y0 + rows, x0 // ncol] += 1
        assert (grid == 1).all(), f"domain {j}: cover counts {np.unique(grid)}"


def test_energy_work_list_ends_with_short_strips():
    """The energy launch's work list (host only): it covers every thermal
    row of every column block exactly once; on the 4096x2048 + 4096x64 domain
    the tall strips (36 rows in FP32, 28 in FP64) outnumber the wavefront
    slots (3072 / 2048), so the list ends with 8-row strips cut from the top
    rows, about 0.6 slots of them; a small domain has 8-row strips only; a
    batch of six 1000x480 + 1000x24 auto-strip domains takes 16-row strips for
    the set (3456 > 3072) and ends with short strips from every member; an
    isothermal member is left out, and mixed precisions are rejected."""
    from paper_1911_10747_amd import poolboil as pb
    P = dict(W.BASE_PARAMS, Tc=0.07, rho_L=6.5, rho_V=0.38, rho_S=19.5)
    cfg = lambda **kw: pb.make_config(**dict(P, **kw))
    for prec, tall, slots in ((1, 36, 3072), (0, 28, 2048)):
        w = pb.thermal_work_list([cfg(nx=4096, ny_fluid=2048, ny_solid=64, precision=prec)])
        _cover(w, [(4096, 2112)])
        rows = w[:, 3]
        assert set(rows) == {tall, 8}
        nshort = int((rows == 8).sum())
        assert (rows[-nshort:] == 8).all() and (rows[:-nshort] == tall).all()
        assert 0.5 * slots <= nshort <= 0.7 * slots, nshort
        assert w[:, 2][rows == 8].min() > w[:, 2][rows == tall].max()     # the top rows
    # explicit 28-row strips in FP32 get the tail too
    w = pb.thermal_work_list([cfg(nx=4096, ny_fluid=2048, ny_solid=64, precision=1, thermal_tile=1)])
    _cover(w, [(4096, 2112)])
    assert set(w[:, 3]) == {28, 8} and w[-1, 3] == 8
    # small domain: 8-row strips, 8 x 53
    w = pb.thermal_work_list([cfg(nx=400, ny_fluid=400, ny_solid=20, precision=1)])
    _cover(w, [(400, 420)])
    assert len(w) == 8 * 53 and set(w[:, 3]) == {8}
    # batch of auto-strip domains, with an isothermal seventh member
    six = [cfg(nx=1000, ny_fluid=480, ny_solid=24, precision=1) for _ in range(6)]
    iso = cfg(nx=300, ny_fluid=100, ny_solid=10, precision=1, flags=pb.PB_ISOTHERMAL)
    w = pb.thermal_work_list(six + [iso])
    _cover(w, [(1000, 504)] * 6)
    assert not (w[:, 0] == 6).any()
    assert set(w[:, 3]) == {16, 8}
    short = w[w[:, 3] == 8]
    assert set(short[:, 0]) == set(range(6)) and (w[-len(short):, 3] == 8).all()
    # explicit strips on the first member decide for the batch
    w = pb.thermal_work_list([cfg(nx=1000, ny_fluid=480, ny_solid=24, precision=1, thermal_tile=4)] + six[1:])
    _cover(w, [(1000, 504)] * 6)
    assert set(w[:, 3]) == {16, 8}
    w = pb.thermal_work_list([cfg(nx=1000, ny_fluid=480, ny_solid=24, precision=1, thermal_tile=6)] + six[1:])
    assert set(w[:, 3]) == {8}
    with pytest.raises(pb.PbError):
        pb.thermal_work_list([six[0], cfg(nx=100, ny_fluid=100, ny_solid=10, precision=0)])


def test_flow_work_list_covers_each_node_once():
    """The flow launch's tiles of one domain (host only): every fluid node is
    in exactly one tile (tiles clipped to the domain); with FP32 storage and
    64x8 or 128x4 tiles the columns past the last full tile go to 32x16
    tiles when that takes fewer tiles, and the list is never longer than
    full-shape tiles over the whole domain; FP64 storage and other shapes
    take no alternate tiles."""
    from paper_1911_10747_amd import poolboil as pb
    P = dict(W.BASE_PARAMS, Tc=0.07, rho_L=6.5, rho_V=0.38, rho_S=19.5)
    cfg = lambda **kw: pb.make_config(**dict(P, **kw))

    def cover(w, nx, ny):
        grid = np.zeros((ny, nx), dtype=np.int32)
        for x0, y0, bw, bh, alt in w:
            assert 0 <= x0 < nx and 0 <= y0 < ny
            grid[y0:y0 + bh, x0:x0 + bw] += 1
        assert (grid == 1).all(), np.unique(grid)

    for prec, tile, nx, ny, n_alt in [
            (1, (64, 8), 77, 45, 3),       # 13 columns past 64: 3 tiles of 32x16 instead of 6 of 64x8
            (1, (64, 8), 132, 40, 3),      # 4 columns past 128
            (1, (64, 8), 100, 40, 0),      # 36 columns past 64: more than 32, no alternate tiles
            (1, (64, 8), 4096, 2048, 0),   # no columns past the last full tile
            (1, (64, 8), 70, 3, 0),        # one row: a 32x16 tile saves nothing
            (1, (128, 4), 200, 64, 12),    # 72 columns past 128: 3 x 4 tiles of 32x16 instead of 16 of 128x4
            (1, (32, 16), 77, 45, 0),      # a 32-wide shape has no alternate shape
            (1, (64, 4), 77, 45, 0),       # 256 threads
            (0, (64, 8), 77, 45, 0)]:      # FP64 storage
        c = cfg(nx=nx, ny_fluid=ny, ny_solid=3, precision=prec, tile_x=tile[0], tile_y=tile[1])
        w = pb.flow_work_list(c)
        cover(w, nx, ny)
        alt = w[w[:, 4] == 1]
        assert len(alt) == n_alt, (tile, nx, ny, len(alt))
        assert (alt[:, 2] == 32).all() and (alt[:, 3] == 16).all()
        assert (w[w[:, 4] == 0][:, 2:4] == tile).all()
        assert len(w) <= -(-nx // tile[0]) * -(-ny // tile[1])
        if n_alt:
            assert alt[:, 0].min() == nx // tile[0] * tile[0]


def test_null_handles_refused_without_gpu():
    """The batch-membership calls and the allocation-free read check their
    handles on the host before any device work."""
    from paper_1911_10747_amd import poolboil as pb
    assert pb.lib.pb_batch_add(None, None) == pb.PB_EINVAL
    assert pb.lib.pb_batch_remove(None, None) == pb.PB_EINVAL
    assert pb.lib.pb_batch_size(None) == -1
    assert pb.lib.pb_batch_step(None, 1) == pb.PB_EINVAL
    assert pb.lib.pb_read_fields_noalloc(None, None, None, None, None, None) == pb.PB_EINVAL
    assert pb.lib.pb_read_fields(None, None, None, None, None, None) == pb.PB_EINVAL
    assert pb.lib.pb_profile_reserve(None, 1) == pb.PB_EINVAL
    assert pb.lib.pb_profile_steps(None, 1, None) == pb.PB_EINVAL
    assert "NULL" in pb.lib.pb_last_error().decode()
