"""Host-side checks of the C-ABI library (no GPU): exports, lattice, transfer model, validation."""
import ctypes
import os
import re

import numpy as np
import pytest

from golden_io import d3q19_ordering, table8

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "lbm355.h")) as fh:
        src = fh.read()
    return sorted(set(re.findall(r"^[\w \*]*?\b(lbm_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    import paper_1111_0922_amd as P
    lib = ctypes.CDLL(P._lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P._lib.EXPORTS) | {"lbm_lattice"} or set(P._lib.EXPORTS) <= set(names)


def test_lattice_matches_golden_ordering():
    import paper_1111_0922_amd as P
    c, w, opp = P.lattice()
    C, W, OPP = d3q19_ordering()
    np.testing.assert_array_equal(c, C)
    np.testing.assert_array_equal(opp, OPP)
    np.testing.assert_array_equal(w, np.array([float(v) for v in W]))


@pytest.mark.parametrize("scheme,key", [("ts", "TS"), ("os_push", "OS"), ("os_pull", "OS"), ("os_nt", "OS-NT"),
                                        ("cg", "CG"), ("swap", "SWAP"), ("aa", "AAP"), ("et", "ET")])
def test_paper_transfer_model_reproduces_table8(scheme, key):
    import paper_1111_0922_amd as P
    full_pdfs, full_bytes, ind_pdfs, ind_idx, ind_bytes = table8()[key]
    assert P.model_bytes(scheme, "direct", model="paper") == full_bytes
    assert P.model_bytes(scheme, "indirect", model="paper") == ind_bytes
    assert full_bytes == 8 * full_pdfs and ind_bytes == 8 * ind_pdfs + 4 * ind_idx


def test_gpu_transfer_model():
    """No write-allocate: TS moves 4q PDFs, OS/AA/ET 2q; IDX 18 (TS, OS), 9 avg (AA), 7 (ET table)."""
    import paper_1111_0922_amd as P
    q = 19
    for prec, s in (("f64", 8), ("f32", 4), ("f16s", 2)):
        assert P.model_bytes("ts", "direct", prec) == 4 * q * s
        for sch in ("os_push", "os_pull", "aa", "et"):
            assert P.model_bytes(sch, "direct", prec) == 2 * q * s
        assert P.model_bytes("ts", "indirect", prec) == 4 * q * s + 72
        assert P.model_bytes("aa", "indirect", prec) == 2 * q * s + 36
        assert P.model_bytes("et", "indirect", prec) == 2 * q * s + 28
    assert P.model_bytes("aa", "indirect", "f32") == 188
    assert P.model_bytes("aa", "indirect", "f16s") == 112
    assert P.model_bytes("cg", "direct", "f64") < 0
    # neighbour ids by rank: one 4-byte cell_of entry where IDX reads 18, the same on direct grids
    for prec, s in (("f64", 8), ("f32", 4), ("f32s", 4)):
        assert P.model_bytes("ts", "indirect", prec, model="gpu_rank") == 4 * q * s + 4
        assert P.model_bytes("os_pull", "indirect", prec, model="gpu_rank") == 2 * q * s + 4
        assert P.model_bytes("aa", "indirect", prec, model="gpu_rank") == 2 * q * s + 2
        assert P.model_bytes("et", "indirect", prec, model="gpu_rank") == 2 * q * s + 4
        assert P.model_bytes("aa", "direct", prec, model="gpu_rank") == 2 * q * s


def test_rank_lookup_query_without_gpu():
    import paper_1111_0922_amd as P
    L = P._lib
    lib = L.load()
    assert lib.lbm_rank_lookup_active(None) == L.LBM_E_ARG
    assert lib.lbm_lattice_block(None) == L.LBM_E_ARG
    g = P.Grid(16, 8, 8, addressing="indirect")
    assert lib.lbm_rank_lookup_active(g._h) == L.LBM_E_STATE
    assert lib.lbm_lattice_block(g._h) == L.LBM_E_STATE


def test_validation_errors_without_gpu():
    import paper_1111_0922_amd as P
    with pytest.raises(P.LbmError):
        P.Grid(8, 8, 8, omega=2.0)
    with pytest.raises(P.LbmError):
        P.Grid(0, 8, 8)
    with pytest.raises(P.LbmError):
        P.Grid(2048, 2048, 1024)       # 2^32 cells
    with pytest.raises(P.LbmError):
        P.Grid(2048, 1024, 1024)       # 2^31 cells: one more than the largest box
    assert P.Grid(2048, 1024, 1023, precision="f16s").n_nodes == 2048 * 1024 * 1023
    with pytest.raises(P.LbmError):
        P.Grid(8, 8, 2, wall_z=True)
    with pytest.raises(P.LbmError):
        P.Grid(8, 8, 8, precision="f16s", f16_scale=0.0)
    g = P.Grid(32, 32, 32, wall_z=True)
    assert g.n_nodes == 32 * 32 * 30
    s = g.sizes("ts")
    assert s.pdf_bytes == s.pdf1_bytes == 19 * s.pitch * 8 and s.pitch % 128 == 0 and s.pitch >= 32 ** 3
    assert g.sizes("aa").pdf1_bytes == 0
    # stepping an unbound grid is refused before any launch
    assert g.lib.lbm_step(g._h, P._lib.AA, P._lib.BGK, 1, None) == P._lib.LBM_E_STATE
    gi = P.Grid(16, 16, 16, addressing="indirect")
    assert gi.sizes("aa").pdf_bytes == 0  # unknown until the index is built
    assert gi.lib.lbm_bind(gi._h, P._lib.AA, None, None, None, None, None) == P._lib.LBM_E_STATE


def test_option_ranges_without_gpu():
    """lbm_set_option validates every option on the host; the pitch pad rounds up to 128 elements."""
    import paper_1111_0922_amd as P
    L = P._lib
    g = P.Grid(64, 8, 8, wall_z=True)
    ok = [(L.OPT_WG_LDS, -1), (L.OPT_WG_LDS, 0), (L.OPT_WG_LDS, 122880), (L.OPT_PAIR, -1), (L.OPT_PAIR, 1),
          (L.OPT_BAND, -1), (L.OPT_BAND, 4096), (L.OPT_ROW_STAGE, 0), (L.OPT_ROW_STAGE, 1),
          (L.OPT_SLAB_ORDER, -1), (L.OPT_SLAB_ORDER, 0), (L.OPT_SLAB_ORDER, 1),
          (L.OPT_RANK_LOOKUP, -1), (L.OPT_RANK_LOOKUP, 0), (L.OPT_RANK_LOOKUP, 1),
          (L.OPT_SOA_BLOCK, -1), (L.OPT_SOA_BLOCK, 0), (L.OPT_SOA_BLOCK, 64), (L.OPT_SOA_BLOCK, 1024),
          (L.OPT_SOA_BLOCK, 65536)]
    for opt, val in ok:
        g.set_option(opt, val)
    bad = [(L.OPT_WG_LDS, -2), (L.OPT_WG_LDS, 122881), (L.OPT_PAIR, 2), (L.OPT_PAIR, -2), (L.OPT_BAND, -2),
           (L.OPT_BAND, 4097), (L.OPT_PITCH_PAD, -1), (L.OPT_PITCH_PAD, (1 << 20) + 1), (99, 0),
           (L.OPT_SLAB_ORDER, 2), (L.OPT_SLAB_ORDER, -2), (L.OPT_RANK_LOOKUP, 2), (L.OPT_RANK_LOOKUP, -2),
           (L.OPT_SOA_BLOCK, 1), (L.OPT_SOA_BLOCK, 32), (L.OPT_SOA_BLOCK, 100), (L.OPT_SOA_BLOCK, 1 << 17),
           (L.OPT_SOA_BLOCK, -2)]
    for opt, val in bad:
        with pytest.raises(P.LbmError):
            g.set_option(opt, val)
    p0 = g.sizes("aa").pitch
    g.set_option(L.OPT_PITCH_PAD, 100)
    assert g.sizes("aa").pitch == p0 + 128
    g.set_option(L.OPT_PITCH_PAD, 0)
    assert g.sizes("aa").pitch == p0


@pytest.mark.parametrize("nx", [100, 128, 8192])
@pytest.mark.parametrize("precision", ["f64", "f32", "f32s", "f16s"])
@pytest.mark.parametrize("scheme", ["aa", "ts", "os_push", "os_pull", "et"])
def test_default_storage_order_of_direct_grids_without_gpu(scheme, precision, nx):
    """On a direct SoA grid the lattice is stored in 1024-cell blocks by default for the two-step,
    one-step and esoteric-twist schemes with 8- and 4-byte storage; the AA pattern with FP64 storage
    in 4096-cell blocks when they hold whole rows (nx divides 4096 or 4096 divides nx); everything
    else in plain SoA.  A blocked lattice's pitch covers whole blocks, a plain one's is the cell count
    rounded to 128.  AoS lattices have no blocks."""
    import paper_1111_0922_amd as P
    ny, nz = 30, 20
    n = nx * ny * nz
    g = P.Grid(nx, ny, nz, wall_z=True, precision=precision, f16_scale=1.0)
    if scheme != "aa":
        b = 1024 if precision != "f16s" else 128
    else:
        b = 4096 if precision == "f64" and (4096 % nx == 0 or nx % 4096 == 0) else 128
    assert g.sizes(scheme).pitch == -(-n // b) * b
    g.set_option(P._lib.OPT_SOA_BLOCK, 0)
    assert g.sizes(scheme).pitch == -(-n // 128) * 128
    g.set_option(P._lib.OPT_SOA_BLOCK, 4096)
    assert g.sizes(scheme).pitch == -(-n // 4096) * 4096
    aos = P.Grid(nx, ny, nz, wall_z=True, layout="aos", precision=precision, f16_scale=1.0)
    aos.set_option(P._lib.OPT_SOA_BLOCK, 4096)
    assert aos.sizes(scheme).pdf_bytes == -(-n * 19 * {"f64": 8, "f16s": 2}.get(precision, 4) // 256) * 256


def test_every_declaration_cites_a_passage_or_says_it_has_none():
    """Each entry point's comment in lbm355.h names the paper passage that defines it (a section,
    table or figure) or says that it has none (an addition of this library)."""
    with open(os.path.join(ROOT, "include", "lbm355.h")) as fh:
        src = fh.read()
    missing = []
    for m in re.finditer(r"^(?:const char \*|int64_t |double |int )(lbm_\w+)\(", src, flags=re.M):
        head = src[:m.start()]
        comment = " ".join(head[head.rfind("/*"):].replace("*", " ").split())
        if not re.search(r"\b(Secs?\.|Tables?|Fig\.)\s*\d|No paper passage|cannot allocate", comment):
            missing.append(m.group(1))
    assert not missing, missing


def test_block_order_and_batch_sync_validation_without_gpu():
    """lbm_set_block_order is refused on a direct grid and before the index exists; lbm_batch_sync and
    lbm_reduce_moments_noalloc refuse null handles; none of these touches the GPU."""
    import paper_1111_0922_amd as P
    L = P._lib
    lib = L.load()
    fake = ctypes.c_void_p(256)
    direct = P.Grid(8, 8, 8)
    assert lib.lbm_set_block_order(direct._h, fake, 1) == L.LBM_E_UNSUPPORTED
    ind = P.Grid(16, 16, 16, addressing="indirect")
    assert lib.lbm_set_block_order(ind._h, fake, 1) == L.LBM_E_STATE
    assert lib.lbm_set_block_order(ind._h, None, 0) == L.LBM_OK      # natural order: always allowed
    assert lib.lbm_set_block_order(None, None, 0) == L.LBM_E_ARG
    assert lib.lbm_batch_sync(None, None, None) == L.LBM_E_ARG
    assert lib.lbm_reduce_moments_noalloc(None, fake, None) == L.LBM_E_ARG
