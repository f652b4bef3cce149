"""Host-side checks of the C ABI (no GPU compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmeqeq.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pq_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_documented_entry_points():
    names = _declared()
    for n in ["pq_create", "pq_set_system", "pq_coulomb", "pq_neighbor_pairs", "pq_qeq_solve",
              "pq_shadow_step", "pq_qeq_vjp", "pq_server_create", "pq_server_submit", "pq_server_poll"]:
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    import paper_2503_21176_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libpmeqeq.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTS) == _declared()
    L = P.load()
    assert L.pq_abi_version() == P.ABI_VERSION == 5
    assert L.pq_coulomb_constant() == 14.3996454784


def test_params_struct_layout_matches_header():
    import paper_2503_21176_amd as P
    # box[3], cutoff, skin, alpha (6 doubles) + grid[3], order, kmax[3], method, flags (9 int32),
    # 4 bytes of padding, tilt[3]
    assert ctypes.sizeof(P.Params) == 6 * 8 + 9 * 4 + 4 + 3 * 8
    assert P.Params.grid.offset == 48 and P.Params.flags.offset == 80 and P.Params.tilt.offset == 88
    assert ctypes.sizeof(P.SolveInfo) == 24


def test_make_params_validation_on_host():
    import paper_2503_21176_amd as P
    p = P.make_params(20.0, 8.0, 0.35, grid=32, order=4)
    assert p.method == P.METHOD_PME and list(p.grid) == [32, 32, 32]
    p = P.make_params([20.0, 21.0, 22.0], 8.0, 0.35, kmax=8, method="ewald")
    assert p.method == P.METHOD_EWALD and list(p.kmax) == [8, 8, 8]
    with pytest.raises(ValueError):
        P.make_params(20.0, 8.0, 0.35, method="p3m")
    # triclinic: rows a, b, c of a lower triangular matrix
    H = [[20.0, 0, 0], [3.0, 21.0, 0], [-2.0, 4.0, 22.0]]
    p = P.make_params(H, 8.0, 0.35, grid=32, order=4)
    assert list(p.box) == [20.0, 21.0, 22.0] and list(p.tilt) == [3.0, -2.0, 4.0]
    assert list(P.make_params(20.0, 8.0, 0.35, grid=32).tilt) == [0.0, 0.0, 0.0]
    with pytest.raises(ValueError):
        P.make_params([[20.0, 1.0, 0], [0, 21.0, 0], [0, 0, 22.0]], 8.0, 0.35, grid=32)


def test_result_and_tune_struct_layouts():
    import paper_2503_21176_amd as P
    # q pointer, energy, solve info (24), status + pad, three doubles, message[256]
    assert P.Result.message.offset == 8 + 8 + 24 + 8 + 24
    assert ctypes.sizeof(P.Result) == 8 + 8 + 24 + 8 + 24 + 256
    assert P.Request.params.offset == 8 + 4 * 8 + 2 * 8 + 4 * 4
    assert ctypes.sizeof(P.Request) == P.Request.params.offset + ctypes.sizeof(P.Params)
    assert ctypes.sizeof(P.TuneResult) == 32 and P.TuneResult.fft_lds_bytes.offset == 24


def test_request_footprint_is_host_only_and_sane():
    # the admission estimate needs no device: positive, growing with the atom
    # count, larger for the FP64 form and for longer GMRES restarts
    import paper_2503_21176_amd as P
    def fp(n, fp64=False, restart=50):
        L = (n / 0.1) ** (1 / 3)
        K = 2 * ((int(L) + 2) // 2)
        return P.request_footprint(n, P.make_params(L, 9.0, 0.29, grid=max(K, 10), order=5, fp64=fp64), restart)
    a, b = fp(1000), fp(20000)
    assert 0 < a < b
    assert fp(20000, fp64=True) > b
    assert fp(20000, restart=200) > b
    with pytest.raises(ValueError):
        P.request_footprint(0, P.make_params(10.0, 4.0, 0.5, grid=10, order=4))


def test_md_cfg_layout_matches_header():
    import paper_2503_21176_amd as P
    # dt, (n_krylov, dissipation), kappa, rep_a, rep_rho, (mode, max_it), (restart, reserved), tol
    assert ctypes.sizeof(P.MdCfg) == 64
    assert P.MdCfg.kappa.offset == 16 and P.MdCfg.mode.offset == 40 and P.MdCfg.tol.offset == 56
