"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/lbm.h, its structs have the layout the
binding assumes, argument errors are reported before any device work, and the
host maths of the weights agree with the oracle."""
import ctypes as C
import math
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2410_13165_amd import lbm as B
from oracle import lbm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_binding_functions():
    assert set(_declared_functions()) == set(B.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbm_[a-z_]+)", out))
    assert set(_declared_functions()) <= exported


_LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "lbm.h"
#define P(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("lbm_params size %zu\n", sizeof(lbm_params));
  printf("lbm_field size %zu\n", sizeof(lbm_field));
  printf("lbm_info_t size %zu\n", sizeof(lbm_info_t));
  P(lbm_params, dx); P(lbm_params, origin); P(lbm_params, u); P(lbm_params, R);
  P(lbm_params, g); P(lbm_params, m4); P(lbm_params, use_m4); P(lbm_params, bc);
  P(lbm_params, bc_order); P(lbm_params, init_order); P(lbm_params, precision);
  P(lbm_params, field); P(lbm_params, alloc); P(lbm_params, free_fn);
  P(lbm_params, alloc_ctx); P(lbm_params, stream); P(lbm_params, wall_data);
  P(lbm_params, steps_per_pass); P(lbm_params, check_every); P(lbm_info_t, steps_per_pass);
  P(lbm_field, n_modes); P(lbm_field, amps); P(lbm_field, kvecs); P(lbm_field, phases);
  P(lbm_field, Rr); P(lbm_field, W); P(lbm_field, center);
  P(lbm_info_t, dims); P(lbm_info_t, nodes); P(lbm_info_t, step); P(lbm_info_t, omega);
  P(lbm_info_t, m4); P(lbm_info_t, min_omega); P(lbm_info_t, s); P(lbm_info_t, dt);
  P(lbm_info_t, phi_ref); P(lbm_info_t, bytes_per_lu); P(lbm_info_t, pstride);
  return 0;
}
"""


def test_struct_layouts_match_the_header():
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "layout.c")
        exe = os.path.join(tmp, "layout")
        open(src, "w").write(_LAYOUT_C)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    py = {"lbm_params": B.LbmParams, "lbm_field": B.LbmField, "lbm_info_t": B.LbmInfo}
    for line in out.splitlines():
        sname, field, val = line.split()
        if field == "size":
            assert C.sizeof(py[sname]) == int(val), sname
        else:
            assert getattr(py[sname], field).offset == int(val), (sname, field)


def test_params_default():
    lib = B.load_library()
    p = B.LbmParams()
    lib.lbm_params_default(C.byref(p))
    assert p.struct_size == C.sizeof(B.LbmParams)
    assert p.dx == 1.0 and p.g == 0.5 and p.bc_order == 4 and p.init_order == 3
    assert p.precision == 0 and [list(b) for b in p.bc] == [[0, 0]] * 4
    assert p.wall_data == 0 and p.steps_per_pass == 2 and p.check_every == 0


def _create(d, dims, tau, **kw):
    lib = B.load_library()
    p = B.LbmParams()
    lib.lbm_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "bc":
            # per axis: one code for both faces, or a (lower, upper) pair
            for a, b in enumerate(v):
                lo, hi = (b, b) if isinstance(b, int) else b
                p.bc[a][0], p.bc[a][1] = lo, hi
        else:
            setattr(p, k, v)
    arr = (C.c_int64 * 4)(*(list(dims) + [1] * (4 - len(dims))))
    h = C.c_void_p()
    rc = lib.lbm_create(d, arr, tau, C.byref(p), C.byref(h))
    return rc, h, lib.lbm_last_error(None).decode()


@pytest.mark.parametrize("args,code,msg", [
    ((0, (4,), 0.5), B.EINVAL, "d must be"),
    ((5, (4,) * 4, 0.5), B.EINVAL, "d must be"),
    ((2, (4, 4), 0.0), B.EINVAL, "tau"),
    ((2, (4, 4), -1.0), B.EINVAL, "tau"),
    ((2, (0, 4), 0.5), B.EINVAL, "dims"),
    ((3, (2048, 2048, 1024), 0.5), B.EINVAL, "2^31"),
])
def test_create_rejects_bad_arguments(args, code, msg):
    rc, h, err = _create(*args)
    assert rc == code and not h.value and msg in err


def test_create_rejects_walls_without_field_and_mixed_schemes():
    rc, h, err = _create(2, (8, 8), 0.5, bc=[1, 1])
    assert rc == B.EINVAL and "field" in err
    rc, h, err = _create(2, (8, 8), 0.5, bc=[1, 2])
    assert rc == B.EUNSUPPORTED and "mixed" in err
    # per-face codes: a periodic face needs a periodic opposite face, and the
    # faces of one axis cannot mix the two schemes either
    rc, h, err = _create(2, (8, 8), 0.5, bc=[(0, 1), 0])
    assert rc == B.EINVAL and "periodic face" in err
    rc, h, err = _create(2, (8, 8), 0.5, bc=[0, (2, 0)])
    assert rc == B.EINVAL and "periodic face" in err
    rc, h, err = _create(2, (8, 8), 0.5, bc=[(1, 2), 0])
    assert rc == B.EUNSUPPORTED and "mixed" in err
    rc, h, err = _create(2, (8, 8), 0.5, bc=[(1, 3), 0])
    assert rc == B.EINVAL and "boundary code" in err
    rc, h, err = _create(2, (1, 8), 0.5, bc=[1, 0])
    assert rc == B.EINVAL and "2 nodes" in err
    rc, h, err = _create(2, (8, 8), 0.5, init_order=2)
    assert rc == B.EINVAL and "init_order" in err
    rc, h, err = _create(2, (8, 8), 0.5, dx=0.0)
    assert rc == B.EINVAL and "dx" in err
    rc, h, err = _create(3, (8, 8, 8), 0.5, steps_per_pass=3)
    assert rc == B.EINVAL and "steps_per_pass" in err
    rc, h, err = _create(3, (8, 8, 8), 0.5, check_every=-1)
    assert rc == B.EINVAL and "check_every" in err


def test_tangential_wall_data_needs_nonzero_normal_velocity():
    lib = B.load_library()
    p = B.LbmParams()
    lib.lbm_params_default(C.byref(p))
    amps = (C.c_double * 1)(1.0)
    kv = (C.c_double * 2)(1.0, 2.0)
    f = B.LbmField()
    f.kind, f.n_modes, f.amps, f.kvecs = 1, 1, amps, kv
    p.field = C.pointer(f)
    p.bc[1][0] = p.bc[1][1] = 1
    p.u[0], p.u[1] = 0.1, 0.0
    p.wall_data = 1
    arr = (C.c_int64 * 4)(8, 8, 1, 1)
    h = C.c_void_p()
    assert lib.lbm_create(2, arr, 0.5, C.byref(p), C.byref(h)) == B.EINVAL
    assert "u_j != 0" in lib.lbm_last_error(None).decode() and not h.value
    p.wall_data = 7
    assert lib.lbm_create(2, arr, 0.5, C.byref(p), C.byref(h)) == B.EINVAL
    assert "wall_data" in lib.lbm_last_error(None).decode()


def test_null_handle_calls_fail_cleanly():
    lib = B.load_library()
    assert lib.lbm_step(None, 1) == B.EINVAL
    assert lib.lbm_moments(None, B.MOM_ALL, None, None) == B.EINVAL
    assert lib.lbm_destroy(None) == B.OK
    assert lib.lbm_state_bytes(None) == -1


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_host_weights_match_oracle(d):
    """The library's closed-form weights (eq. omega_k-2 with eq. meq-4rd) against
    the oracle's M^{-1} eps."""
    rng = np.random.default_rng(70 + d)
    for _ in range(25):
        u = rng.uniform(-0.6, 0.6, d)
        w, m4, mn = B.equilibrium_weights(u)
        np.testing.assert_allclose(w, O.omega(u), rtol=0, atol=1e-14)
        if d >= 2:
            assert abs(m4 - O.m4_interpolated(u)) < 1e-15
        assert abs(mn - O.min_omega(u)) < 1e-14
        m4x = float(rng.uniform(-0.1, 0.2))
        w2, m42, _ = B.equilibrium_weights(u, m4=m4x)
        if d >= 2:
            np.testing.assert_allclose(w2, O.omega(u, m4=m4x), rtol=0, atol=1e-14)
            assert m42 == m4x


def test_host_weights_reject_bad_dimension():
    with pytest.raises(B.LbmError):
        B.equilibrium_weights([0.1] * 5)


def test_stability_map_rejects_bad_arguments_before_any_launch():
    lib = B.load_library()
    z = None
    cases = [
        ((0, 1, z, z, 0.5, 8), "d must be"),
        ((5, 1, z, z, 0.5, 8), "d must be"),
        ((2, -1, z, z, 0.5, 8), "count"),
        ((2, 1, z, z, 0.5, 0), "m must be"),
        ((2, 1, z, z, 0.5, (1 << 20) + 1), "m must be"),
        ((4, 1, z, z, 0.5, 1024), "m\\^d"),
        ((2, 1, z, z, math.inf, 8), "g must be"),
        ((2, 3, z, z, 0.5, 8), "must not be null"),
    ]
    for (d, count, sig, s, g, m), msg in cases:
        rc = lib.lbm_stability_map(d, count, sig, s, g, m, None, None, None, None)
        assert rc == B.EINVAL
        assert re.search(msg, lib.lbm_last_error(None).decode())
    # nothing to do: success without touching a device
    assert lib.lbm_stability_map(2, 0, None, None, 0.5, 8, None, None, None, None) == B.OK


def test_build_compiles_every_source_once():
    from paper_2410_13165_amd import build
    on_disk = sorted(f for f in os.listdir(build.CSRC) if f.endswith(".hip"))
    assert sorted(build.SOURCES) == on_disk
    cmd = build.compile_command(build.SOURCES[0], "x.o")
    assert "--offload-arch=gfx950" in cmd and "-packed-fp32-ops" in cmd and "-c" in cmd
    # the d = 3 and d = 4 wall units keep their parameter block out of scratch
    for src in ("walls_d3.hip", "walls_d3t.hip", "walls_d4.hip", "walls_d4t.hip"):
        assert "-instcombine-max-copied-from-constant-users=4000" in build.compile_command(src, "x.o")
