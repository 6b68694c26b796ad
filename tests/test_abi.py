"""The C ABI library loads, exports every symbol include/lbm_stefan.h
declares, and its host-side argument checks work (no GPU needed: these
paths return before any HIP call)."""
import ctypes
import os
import re
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_stefan.h")


@pytest.fixture(scope="module")
def L():
    from paper_2505_13097_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2505_13097_amd import build
        build.build(verbose=False)
    return _lib


def declared_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_stefan_\w+)\s*\(", text)))


def test_header_symbols_exported(L):
    names = declared_functions(HEADER)
    assert "lbm_stefan_init" in names and "lbm_stefan_step" in names
    lib = L.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares the same set
    assert set(L.SIGNATURES) <= set(names)


def test_version_string(L):
    v = L.lib().lbm_stefan_version().decode()
    assert "gfx950" in v


def _params(L, prob, **over):
    from paper_2505_13097_amd.stefan import make_params
    p, keep = make_params(prob)
    for k, v in over.items():
        setattr(p, k, v)
    return p, keep


def _ws(L, p):
    n = ctypes.c_size_t()
    rc = L.lib().lbm_stefan_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    return rc, n.value


@pytest.mark.parametrize("field,value", [
    ("tau", 0.5), ("tau", 0.3), ("ste", 0.0), ("ste", -1.0), ("delta", 0.0),
    ("newton_tol", 0.0), ("newton_max_it", 0), ("newton_max_it", 1001),
    ("nx", 2), ("ny", 2), ("q", 4), ("dim", 3), ("storage", 7),
    ("newton_mode", 5), ("variant", 99), ("tau", float("nan")),
    ("scheme", 3), ("scheme", -1),
])
def test_invalid_params_rejected(L, field, value):
    p, keep = _params(L, synth.planar_2d(n=32, ny=16))
    setattr(p, field, value)
    rc, _ = _ws(L, p)
    assert rc == L.EINVAL
    msg = L.lib().lbm_stefan_last_error(None).decode()
    assert msg and msg != "no error"


def test_lattice_dimension_mismatch(L):
    p, _ = _params(L, synth.stefan_1d(nx=32))
    p.ny = 4
    assert _ws(L, p)[0] == L.EINVAL
    p, _ = _params(L, synth.planar_2d(n=32, ny=16))
    p.bc[2] = L.BC_DIRICHLET       # y- not periodic, y+ periodic
    assert _ws(L, p)[0] == L.EINVAL


@pytest.mark.parametrize("maker,q,s", [
    (lambda: synth.stefan_1d(nx=256), 3, 8),
    (lambda: synth.planar_2d(n=128, ny=96), 5, 4),
    (lambda: synth.cavity_2d(n=200, ny=130), 9, 4),
])
def test_workspace_holds_two_state_buffers(L, maker, q, s):
    prob = maker()
    p, _ = _params(L, prob)
    rc, n = _ws(L, p)
    assert rc == L.OK
    assert n >= 2 * q * prob.nodes * s
    assert n < 2 * q * prob.nodes * s + 64 * prob.nodes + (1 << 20)
    p.flags = L.FLAG_ADJOINT
    rc, n2 = _ws(L, p)
    assert rc == L.OK and n2 >= n


def test_init_rejects_small_or_misaligned_workspace(L):
    p, _ = _params(L, synth.planar_2d(n=32, ny=16))
    rc, n = _ws(L, p)
    h = ctypes.c_void_p()
    lib = L.lib()
    assert lib.lbm_stefan_init(ctypes.byref(p), None, None, n, None,
                               ctypes.byref(h)) == L.EINVAL
    assert lib.lbm_stefan_init(ctypes.byref(p), None, ctypes.c_void_p(256),
                               n - 1, None, ctypes.byref(h)) == L.EINVAL
    assert lib.lbm_stefan_init(ctypes.byref(p), None, ctypes.c_void_p(4096 + 8),
                               n, None, ctypes.byref(h)) == L.EINVAL
    assert not h.value


def test_variants_listed(L):
    from paper_2505_13097_amd import variant_names
    for q in (3, 5, 9):
        names = variant_names(q)
        assert len(names) >= 3
        assert all(re.fullmatch(r"\d+x\d+(/npt\d|/t2s?)(/r\d+)?(/nt)?(/rev)?", n)
                   or (q == 3 and n == "resident2048") for n in names)
    # D1Q3 only: the resident variant, last in its list
    assert variant_names(3)[-1] == "resident2048"
    assert "resident2048" not in variant_names(5) + variant_names(9)
    assert L.lib().lbm_stefan_variant_name(5, 1, 999) == b""


def test_tape_bytes(L):
    p, _ = _params(L, synth.adjoint_2d(n=64, ny=32))
    n = ctypes.c_size_t()
    lib = L.lib()
    assert lib.lbm_stefan_tape_bytes(ctypes.byref(p), 0, 8, ctypes.byref(n)) == L.EINVAL
    assert lib.lbm_stefan_tape_bytes(ctypes.byref(p), 100, 0, ctypes.byref(n)) == L.EINVAL
    assert lib.lbm_stefan_tape_bytes(ctypes.byref(p), 100, 10, ctypes.byref(n)) == L.OK
    state = 5 * 64 * 32 * 4
    assert n.value >= (10 + 1 + 10) * state


def test_batch_rejects_mixed_lattices(L):
    from paper_2505_13097_amd.stefan import make_params
    a, _ = make_params(synth.planar_2d(n=64, ny=32))
    b, _ = make_params(synth.cavity_2d(n=64, ny=32))
    arr = (L.Params * 2)(a, b)
    n = ctypes.c_size_t()
    assert L.lib().lbm_stefan_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == L.EINVAL
    arr = (L.Params * 2)(a, a)
    assert L.lib().lbm_stefan_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == L.OK
    assert n.value >= 2 * 2 * 5 * 64 * 32 * 4


def test_eebm_rejects_reverse_mode(L):
    p, _ = _params(L, synth.planar_2d(n=32, ny=16), scheme=L.SCHEME_EEBM)
    assert _ws(L, p)[0] == L.OK
    p.flags = L.FLAG_ADJOINT
    assert _ws(L, p)[0] == L.EINVAL
    assert b"IREBM" in L.lib().lbm_stefan_last_error(None)


def test_batch_rejects_mixed_schemes(L):
    from paper_2505_13097_amd.stefan import make_params
    a, _ = make_params(synth.planar_2d(n=64, ny=32))
    b, _ = make_params(synth.planar_2d(n=64, ny=32).with_(scheme="eebm"))
    assert b.scheme == L.SCHEME_EEBM
    n = ctypes.c_size_t()
    arr = (L.Params * 2)(a, b)
    assert L.lib().lbm_stefan_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == L.EINVAL
    arr = (L.Params * 2)(b, b)
    assert L.lib().lbm_stefan_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == L.OK


def test_ctypes_structs_match_header(L, tmp_path):
    """Size and field offsets of the binding's structs equal the C ones."""
    fields = [f for f, _ in L.Params._fields_]
    sfields = [f for f, _ in L.Stats._fields_]
    src = ["#include <stddef.h>", "#include <stdio.h>",
           '#include "lbm_stefan.h"', "int main(void) {",
           '  printf("%zu\\n", sizeof(lbm_stefan_params));',
           '  printf("%zu\\n", sizeof(lbm_stefan_stats));']
    src += [f'  printf("%zu\\n", offsetof(lbm_stefan_params, {f}));'
            for f in fields]
    src += [f'  printf("%zu\\n", offsetof(lbm_stefan_stats, {f}));'
            for f in sfields]
    src += ["  return 0;", "}"]
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o",
                    str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True,
                                          text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(L.Params), ctypes.sizeof(L.Stats)]
    want += [getattr(L.Params, f).offset for f in fields]
    want += [getattr(L.Stats, f).offset for f in sfields]
    assert out == want


def test_neumann_wall_rules(L):
    """Neumann walls (eq. Neu_on_q): not beside bounce-back walls, no
    reverse mode, not in the batched form."""
    from paper_2505_13097_amd.stefan import make_params
    prob = synth.freezing_cavity_2d(n=33, q=9)
    p, _ = _params(L, prob)
    assert p.bc[1] == L.BC_NEUMANN and _ws(L, p)[0] == L.OK
    p.bc[2] = L.BC_BOUNCEBACK
    p.bc[3] = L.BC_BOUNCEBACK
    assert _ws(L, p)[0] == L.EINVAL
    assert b"bounce-back" in L.lib().lbm_stefan_last_error(None)
    p, _ = _params(L, prob, flags=L.FLAG_ADJOINT)
    assert _ws(L, p)[0] == L.EINVAL
    p.bc[4 - 3] = L.BC_NEUMANN + 1
    assert _ws(L, p)[0] == L.EINVAL
    a, _ = make_params(prob)
    n = ctypes.c_size_t()
    arr = (L.Params * 2)(a, a)
    assert L.lib().lbm_stefan_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == L.EINVAL
    assert b"Neumann" in L.lib().lbm_stefan_batch_last_error(None)


def test_ilfbm_rules_and_workspace(L):
    """ILFBM (Algorithm 1): three more liquid fraction planes in the
    workspace, no reverse mode, not in the batched form."""
    from paper_2505_13097_amd.stefan import make_params
    prob = synth.planar_2d(n=64, ny=32)
    p, _ = _params(L, prob)
    rc, n_irebm = _ws(L, p)
    p.scheme = L.SCHEME_ILFBM
    rc, n_ilfbm = _ws(L, p)
    assert rc == L.OK and n_ilfbm >= n_irebm + 3 * 8 * prob.nodes
    p.flags = L.FLAG_ADJOINT
    assert _ws(L, p)[0] == L.EINVAL
    a, _ = make_params(prob.with_(scheme="ilfbm"))
    n = ctypes.c_size_t()
    arr = (L.Params * 2)(a, a)
    assert L.lib().lbm_stefan_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == L.EINVAL


def test_3d_rules_and_workspace(L):
    """D3Q7 / D3Q19: accepted with z faces of their own; workspace holds two
    state buffers of q * nx * ny * nz values; the 3D restrictions return
    EINVAL."""
    for q in (7, 19):
        prob = synth.cavity_3d(n=40, ny=24, nz=17, q=q)
        p, _ = _params(L, prob)
        rc, n = _ws(L, p)
        assert rc == 0
        assert n >= 2 * q * 40 * 24 * 17 * 4
        for field, value in (("nz", 2), ("q", 9), ("scheme", L.SCHEME_ILFBM),
                             ("flags", L.FLAG_ADJOINT), ("variant", 99)):
            p, _ = _params(L, prob)
            setattr(p, field, value)
            assert _ws(L, p)[0] == L.EINVAL, (q, field)
        p, _ = _params(L, prob)
        p.bc_z[1] = L.BC_PERIODIC          # one periodic z face
        assert _ws(L, p)[0] == L.EINVAL
        p, _ = _params(L, prob)
        p.bc_z[0] = L.BC_NEUMANN           # beside bounce-back y walls
        assert _ws(L, p)[0] == L.EINVAL
        p, _ = _params(L, synth.freezing_cube_3d(n=9, q=q))
        assert _ws(L, p)[0] == 0
        p.bc_z[1] = 7
        assert _ws(L, p)[0] == L.EINVAL
    # wall profiles are 2D only
    import numpy as np
    prob = synth.cavity_3d(n=16, q=7).with_(
        wall_profile=(np.ones(16), None, None, None))
    p, keep = _params(L, prob)
    assert _ws(L, p)[0] == L.EINVAL
    # 2^31 nodes or more
    p, _ = _params(L, synth.cavity_3d(n=16, q=7))
    p.nx, p.ny, p.nz = 2048, 1024, 1024
    assert _ws(L, p)[0] == L.EINVAL
    # the batched form refuses 3D instances
    a, _ = _params(L, synth.cavity_3d(n=16, q=7))
    arr = (L.Params * 2)(a, a)
    n = ctypes.c_size_t()
    assert L.lib().lbm_stefan_batch_workspace_bytes(
        arr, 2, ctypes.byref(n)) == L.EINVAL
    assert "1D and 2D" in L.lib().lbm_stefan_batch_last_error(None).decode()


def test_3d_variants_listed(L):
    """Every 3D variant fits the kernel's launch bound (256 threads) with
    whole waves along x: block = (tile_x / npt) x tile_y threads."""
    import re
    from paper_2505_13097_amd import variant_names
    for q in (7, 19):
        names = variant_names(q, "f32")
        assert len(names) >= 8
        for n in names:
            m = re.fullmatch(r"(\d+)x(\d+)/npt(\d+)/z(\d+)(/nt)?(/s)?", n)
            assert m, n
            tx, ty, npt, cz = (int(m.group(k)) for k in range(1, 5))
            bx = tx // npt
            assert bx % 64 == 0 and bx * ty <= 256 and cz >= 1, n


def test_step_noalloc_refusals(L):
    """lbm_stefan_step_noalloc refuses, before any device call, what it
    cannot run in its fixed scratch: NULL or equal buffers, wall profiles,
    ILFBM, the reverse mode, and lattices whose statistics slots and energy
    partials exceed LBM_STEFAN_NOALLOC_SCRATCH_BYTES (the buffer pointers
    are never dereferenced on these paths)."""
    import numpy as np
    lib = L.lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)

    def call(prob, src=a, dst=b, **over):
        p, keep = _params(L, prob, **over)
        rc = lib.lbm_stefan_step_noalloc(ctypes.byref(p), src, dst, None, None)
        return rc, lib.lbm_stefan_last_error(None).decode()

    prob = synth.planar_2d(n=64, ny=32)
    assert call(prob, src=None)[0] == L.EINVAL
    assert call(prob, dst=a)[0] == L.EINVAL
    assert call(prob, scheme=L.SCHEME_ILFBM)[0] == L.EINVAL
    assert call(prob, flags=L.FLAG_ADJOINT)[0] == L.EINVAL
    assert call(prob, tau=0.5)[0] == L.EINVAL
    rc, msg = call(prob.with_(wall_profile=(np.ones(32), None, None, None)))
    assert rc == L.EINVAL and "profile" in msg
    # 8192 x 8192 D2Q9 fits (131072 slots of 32 B, 32768 partials); a
    # 40000 x 40000 lattice needs 3.1 M slots, about 100 MB
    rc, msg = call(synth.cavity_2d(n=40000))
    assert rc == L.EINVAL and "fixed scratch" in msg
    rc, msg = call(synth.cavity_3d(n=1024, ny=1024, nz=1536, q=7))
    assert rc == L.EINVAL and "fixed scratch" in msg
