"""CPU tests of libcgp's host side: exported symbols, host-only topology
(bit-exact against the oracle), and argument / mesh validation errors.
No GPU compute is called here."""
import re
from pathlib import Path

import numpy as np
import pytest

import workloads as W

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def cgp():
    import paper_1610_06993_amd as m
    m.lib()
    return m


def test_library_exports_every_declared_symbol(cgp):
    header = (ROOT / "include" / "cgp.h").read_text()
    names = set(re.findall(r"^(?:cgp_status|int32_t|void|const char\s*\*)\s*\*?\s*(cgp_[a-z_0-9]+)\s*\(", header, re.M))
    assert {"cgp_mesh_create", "cgp_assemble", "cgp_step", "cgp_poisson_solve"} <= names
    L = cgp.lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert cgp.abi_version() == int(re.search(r"CGP_ABI_VERSION (\d+)", header).group(1))
    # every function that takes arguments has a ctypes prototype: an undeclared pointer argument
    # would be passed as a 32-bit int
    decls = dict(re.findall(r"^(?:cgp_status|int32_t|void|const char\s*\*)\s*\*?\s*(cgp_[a-z_0-9]+)\s*\(([^)]*)\)",
                            header, re.M))
    undeclared = [n for n, args in decls.items() if args.strip() not in ("", "void") and getattr(L, n).argtypes is None]
    assert not undeclared, undeclared


TOPO = ["xy", "tri", "bedge", "bkind", "edges", "rowptr_f", "col_f", "slot_f", "colour_f", "rowptr_c", "col_c",
        "slot_c", "colour_c", "vdir", "pdir"]


@pytest.mark.parametrize("which,levels", [("tg", 1), ("tg", 0), ("bfs", 2), ("cyl", 1), ("cyl", 3)])
def test_topology_bit_exact_against_oracle(cgp, orc, which, levels):
    mesh = {"tg": lambda: W.unit_square_tg(12), "bfs": lambda: W.bfs_channel(40, 6),
            "cyl": lambda: W.cylinder_channel(4000, seed=5)}[which]()
    g = cgp.Mesh(mesh, levels, host_only=True)
    o = orc.Problem(mesh, levels)
    assert g.info == {k: v for k, v in o.info.items()}
    for lv in range(levels + 1):
        for k in ("xy", "tri", "bedge", "bkind", "edges") + (("parent",) if lv else ()):
            a, b = g.export(k, lv), o.export(k, lv)
            assert a.dtype == b.dtype and np.array_equal(a, b), (k, lv)
    for k in TOPO[5:]:
        assert np.array_equal(g.export(k), o.export(k)), k


def test_colour_classes_are_node_disjoint(cgp):
    g = cgp.Mesh(W.cylinder_channel(20000, seed=8), 1, host_only=True)
    tri, col = g.export("tri"), g.export("colour_f")
    for c in range(col.max() + 1):
        nodes = tri[col == c].ravel()
        assert len(np.unique(nodes)) == len(nodes)


def _expect(cgp, status, fn):
    with pytest.raises(cgp.CGPError) as e:
        fn()
    assert e.value.status == status, str(e.value)


def test_invalid_meshes_rejected(cgp):
    base = W.unit_square_tg(4)

    def clone(**kw):
        m = W.CoarseMesh(base.xy.copy(), base.tri.copy(), base.bedge.copy(), base.bkind.copy())
        for k, v in kw.items():
            setattr(m, k, v)
        return m

    cw = clone()
    cw.tri[0, [1, 2]] = cw.tri[0, [2, 1]]
    _expect(cgp, 2, lambda: cgp.Mesh(cw, 1, host_only=True))
    untagged = clone(bedge=base.bedge[1:].copy(), bkind=base.bkind[1:].copy())
    _expect(cgp, 2, lambda: cgp.Mesh(untagged, 1, host_only=True))
    nonman = clone(tri=np.concatenate([base.tri, base.tri[:1]]))
    _expect(cgp, 2, lambda: cgp.Mesh(nonman, 1, host_only=True))
    badkind = clone()
    badkind.bkind[0] = 7
    _expect(cgp, 2, lambda: cgp.Mesh(badkind, 1, host_only=True))
    oob = clone()
    oob.tri[3, 0] = 10_000
    _expect(cgp, 2, lambda: cgp.Mesh(oob, 1, host_only=True))
    _expect(cgp, 1, lambda: cgp.Mesh(base, 9, host_only=True))


def test_host_only_mesh_refuses_device_calls(cgp):
    g = cgp.Mesh(W.unit_square_tg(4), 1, host_only=True)
    _expect(cgp, 7, lambda: g.assemble(1.0, 0.01, 1e-3))
    _expect(cgp, 1, lambda: g.assemble(-1.0, 0.01, 1e-3))
    with pytest.raises(cgp.CGPError):
        g.export("M_f")


def test_persistent_grid_and_spin_limits_validated(cgp):
    """The persistent Poisson kernel needs every block resident at once: more than one block per compute
    unit (at most 256 on a gfx950 part; a host-only mesh has no device to ask) is rejected, as is a
    barrier spin limit outside 2^1..2^30.  The graph switch of the fused PCG is 0 or 1, off by default."""
    g = cgp.Mesh(W.unit_square_tg(4), 1, host_only=True)
    before = g.get_tuning()
    assert before["pcg_graph"] == 0
    for kw in ({"pcg_grid": 257}, {"pcg_grid": 512}, {"pcg_grid": -1}, {"pcg_spin_log2": 31},
               {"pcg_spin_log2": -2}, {"pcg_graph": 2}, {"pcg_graph": -1}):
        _expect(cgp, 1, lambda: g.set_tuning(**kw))
        assert g.get_tuning() == before
    g.set_tuning(pcg_grid=256, pcg_spin_log2=1)
    t = g.get_tuning()
    assert t["pcg_grid"] == 256 and t["pcg_spin_log2"] == 1


def test_paper_prolongation_loop_count_through_the_library(cgp):
    """Section 3.2 / Table 5: the 102400:1600 backward-step resolution needs 68659 prolongation loops,
    the nodes of the two intermediate and the finest meshes.  A step-shaped channel of 800 unit cells
    (94 x 10 cells without a 20 x 7 corner: 1600 triangles, 905 nodes, like the paper's coarse mesh)
    subdivided three times by the library gives the same counts."""
    nx, ny, cx, cy = 94, 10, 20, 7
    keep = np.ones((ny, nx), bool)
    keep[:cy, :cx] = False  # the step's corner below the inlet section
    ids = -np.ones((ny + 1, nx + 1), np.int64)
    used = np.zeros_like(ids, bool)
    for j in range(ny):
        for i in range(nx):
            if keep[j, i]:
                used[j:j + 2, i:i + 2] = True
    ids[used] = np.arange(used.sum())
    J, I = np.nonzero(used)
    xy = np.stack([I, J], 1).astype(np.float64)[np.argsort(ids[used])]
    tris = []
    for j in range(ny):
        for i in range(nx):
            if keep[j, i]:
                a, b, c, d = ids[j, i], ids[j, i + 1], ids[j + 1, i + 1], ids[j + 1, i]
                tris += [(a, b, c), (a, c, d)]
    tri = np.array(tris, np.int32)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = np.sort(e, 1)
    u, inv, cnt = np.unique(key[:, 0] * 100000 + key[:, 1], return_inverse=True, return_counts=True)
    bedge = e[cnt[inv] == 1].astype(np.int32)
    mesh = W.CoarseMesh(xy, tri, bedge, np.ones(len(bedge), np.int32))
    assert mesh.n_nodes == 905 and mesh.n_tris == 1600
    g = cgp.Mesh(mesh, 3, host_only=True)
    sizes = [g.sizes(k) for k in range(4)]
    assert sizes[3]["t"] == 102400
    assert sum(s["n"] for s in sizes[1:]) == 68659
