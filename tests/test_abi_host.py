"""CPU tests of the C ABI: the library loads and exports every declared
symbol; the host-side setup (no GPU calls) agrees with the oracle on counts
and node coordinates; argument and call-order errors are reported."""
import os
import re

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1610_05023_amd", "libdghabc.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dghabc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dgh_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(LIB)
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("n,N,P,bc", [(3, 2, 2, ("habc",) * 6), (4, 3, 3, ("habc",) * 6),
                                      (3, 4, 6, ("habc", "habc", "dirichlet", "habc", "abc", "habc"))])
def test_host_setup_matches_oracle(n, N, P, bc):
    from oracle.solver import Oracle
    from paper_1610_05023_amd import Solver
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    o = Oracle(VX, E, N, P, np.ones(K), np.ones(K), face_bc=bc)
    s = Solver(VX, E, N, P, np.ones(K), np.ones(K), face_bc=bc)
    k = s.counts
    assert (k["K"], k["Ktri"], k["Klin"], k["Kpnt"]) == (o.m.K, o.m.Ktri, o.m.Klin, o.m.Kpnt)
    assert s.shapes() == o.shapes()
    assert np.abs(s.node_coords() - o.node_coords()).max() < 1e-14


def test_general_mesh_inputs():
    """The unstructured test mesh: every element positively oriented, the
    boundary vertices where the Kuhn mesh has them, every face shared by two
    elements or lying on a box plane; the host setup (general element order)
    agrees with the oracle on counts, shapes and node coordinates."""
    from oracle.solver import Oracle
    from paper_1610_05023_amd import Solver
    n = 4
    VX0, E0 = w.kuhn_mesh(n)
    VX, E = w.general_mesh(n, amp=0.1, seed=5)
    assert VX.shape == VX0.shape and E.shape == E0.shape
    on_bnd = np.any((VX0 < 1e-12) | (VX0 > 1 - 1e-12), axis=1)
    assert np.array_equal(VX[on_bnd], VX0[on_bnd])
    assert np.abs(VX[~on_bnd] - VX0[~on_bnd]).max() > 0.01 / n
    d = VX[E[:, 1:]] - VX[E[:, :1]]
    assert np.linalg.det(d).min() > 0
    assert not np.array_equal(np.sort(E, axis=1), np.sort(E0, axis=1))
    assert sorted(map(tuple, np.sort(E, axis=1))) == sorted(map(tuple, np.sort(E0, axis=1)))
    faces = {}
    for e in range(E.shape[0]):
        for f in range(4):
            key = tuple(sorted(np.delete(E[e], f)))
            faces[key] = faces.get(key, 0) + 1
    for key, cnt in faces.items():
        if cnt == 1:
            x = VX[list(key)]
            assert np.any(np.all((x < 1e-12) | (x > 1 - 1e-12), axis=0)), key
        else:
            assert cnt == 2, key
    K = E.shape[0]
    o = Oracle(VX, E, 3, 2, np.ones(K), np.ones(K))
    s = Solver(VX, E, 3, 2, np.ones(K), np.ones(K))
    k = s.counts
    assert (k["K"], k["Ktri"], k["Klin"], k["Kpnt"]) == (o.m.K, o.m.Ktri, o.m.Klin, o.m.Kpnt)
    assert s.shapes() == o.shapes()
    assert np.abs(s.node_coords() - o.node_coords()).max() < 1e-14


def test_state_size_limit():
    """The kernels address a shot's 3D state with 32-bit byte offsets: a
    70^3 x 6 = 2,058,000-tet mesh fits at N = 5 (3.69 GB per 3D array) and
    is refused at N = 6 (6.9 GB)."""
    from paper_1610_05023_amd import Solver, DghError
    VX, E = w.kuhn_mesh(70)
    K = E.shape[0]
    s5 = Solver(VX, E, 5, 0, np.ones(K), np.ones(K))
    assert s5.workspace_size() > 2 * K * 4 * 56 * 8
    s6 = Solver(VX, E, 6, 0, np.ones(K), np.ones(K))
    with pytest.raises(DghError, match="4 GiB"):
        s6.workspace_size()


def test_kuhn_counts():
    from paper_1610_05023_amd import Solver
    n = 5
    VX, E = w.kuhn_mesh(n)
    s = Solver(VX, E, 2, 2, np.ones(E.shape[0]), np.ones(E.shape[0]))
    k = s.counts
    assert (k["Ktri"], k["Klin"], k["Kpnt"]) == (12 * n * n, 12 * n, 8)


def test_errors_reported():
    from paper_1610_05023_amd import Solver, DghError
    VX, E = w.kuhn_mesh(2)
    K = E.shape[0]
    with pytest.raises(DghError, match="EINVAL"):
        Solver(VX, E, 9, 1, np.ones(K), np.ones(K))          # degree out of range
    with pytest.raises(DghError, match="EINVAL"):
        Solver(VX, E, 2, 13, np.ones(K), np.ones(K))         # HABC order out of range
    with pytest.raises(DghError, match="EINVAL"):
        Solver(VX, E, 2, 1, -np.ones(K), np.ones(K))         # negative density
    bad = E.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]                           # inverted tet
    with pytest.raises(DghError, match="EINVAL"):
        Solver(VX, bad, 2, 1, np.ones(K), np.ones(K))
    s = Solver(VX, E, 2, 1, np.ones(K), np.ones(K))
    with pytest.raises(DghError, match="ESTATE"):
        s.step(1, 1e-3)                                       # before bind
    with pytest.raises(DghError, match="ENOMEM"):
        s._call("dgh_bind_workspace", None, 16, None)         # workspace too small


def test_shot_count_and_workspace():
    """n_shots is range-checked at creation; the workspace grows with the
    number of shots by the per-shot state (the shared constants stay)."""
    from paper_1610_05023_amd import Solver, DghError
    VX, E = w.kuhn_mesh(3)
    K = E.shape[0]
    for bad in (0, 4097):
        with pytest.raises(DghError, match="dgh_create"):
            Solver(VX, E, 2, 2, np.ones(K), np.ones(K), n_shots=bad)
    sizes = [Solver(VX, E, 2, 2, np.ones(K), np.ones(K), n_shots=k).workspace_size()
             for k in (1, 2, 5)]
    assert sizes[1] > sizes[0] and abs((sizes[2] - sizes[1]) - 3 * (sizes[1] - sizes[0])) < 4096
    s = Solver(VX, E, 2, 2, np.ones(K), np.ones(K), n_shots=2)
    assert s.counts["n_shots"] == 2
