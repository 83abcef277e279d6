"""The C interface without a GPU: the library loads, exports every function
include/xs.h declares, its structs match the binding's layouts, and host-side
validation rejects bad tables and arguments before any device call."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth
from paper_2402_09222_amd import xs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(xs.LIB_PATH):
        from paper_2402_09222_amd import build
        build.build()
    return xs.load_library()


def test_exports_every_declared_function(lib):
    names = xs.declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", xs.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(names) <= exported


STRUCTS = ["xs_table_desc", "xs_params", "xs_table_info_t", "xs_profile_t",
           "xs_tune_config", "xs_tune_result", "xs_tune_request",
           "xs_tune_key", "xs_request",
           "xs_request_stats", "xs_event_config", "xs_event_buffers",
           "xs_event_result", "xs_debug_info"]


def test_struct_layouts_match_header(tmp_path):
    """Size and every field offset of each struct the binding declares equal
    what a C compiler makes of include/xs.h."""
    lines = []
    for name in STRUCTS:
        cls = getattr(xs, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"xs.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) +
                   "\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"),
                    "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True,
                         check=True).stdout.splitlines()
    got = {tuple(l.split()[:-1]): int(l.split()[-1]) for l in out}
    for name in STRUCTS:
        cls = getattr(xs, name)
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def test_status_strings(lib):
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert xs.xs_status_string(st).startswith("XS_")
    assert "unknown" in xs.xs_status_string(-99)


def test_params_default(lib):
    p = xs.xs_params_default(xs.XS_FP32)
    assert p.precision == xs.XS_FP32
    assert p.grid == xs.XS_AUTO and p.sort == xs.XS_AUTO
    assert p.block_size == 0 and p.lookups_per_thread == 0
    assert p.sort_threshold == -1 and p.unroll == 0
    with pytest.raises(xs.XsError) as e:
        xs.xs_params_default(7)
    assert e.value.status == xs.XS_EINVAL


def _small():
    return synth.random_tables(5, 3, [4, 5, 6], 2, sizes=[2, 3])


def _create_status(t, flags=0, bins=0, **over):
    desc, keep = xs.make_desc(t, flags, bins)
    for k, v in over.items():
        setattr(desc, k, v)
    h = ctypes.c_void_p()
    st = xs.load_library().xs_create_tables(ctypes.byref(desc), None,
                                            ctypes.byref(h))
    return st, xs.xs_last_error(), h


def _mutated(**arrays):
    t = _small()
    d = dict(grid_offsets=t.grid_offsets.copy(), energy=t.energy.copy(),
             xs=t.xs.copy(), mat_offsets=t.mat_offsets.copy(),
             mat_nuclides=t.mat_nuclides.copy(), mat_density=t.mat_density.copy())
    for k, fn in arrays.items():
        fn(d[k])
    return synth.Tables(**d)


def _set(i, v):
    def f(a):
        a.reshape(-1)[i] = v
    return f


BAD_TABLES = {
    "energy_not_increasing": dict(energy=_set(1, 1e-5)),
    "energy_nan": dict(energy=_set(2, np.nan)),
    "energy_negative": dict(energy=_set(0, -1.0)),
    "energy_zero": dict(energy=_set(0, 0.0)),
    "energy_below_range": dict(energy=_set(0, 2.0 ** -401)),
    "energy_above_range": dict(energy=_set(-1, 2.0 ** 401)),
    "xs_negative": dict(xs=_set(7, -0.5)),
    "xs_inf": dict(xs=_set(3, np.inf)),
    "density_zero": dict(mat_density=_set(0, 0.0)),
    "density_nan": dict(mat_density=_set(1, np.nan)),
    "nuclide_out_of_range": dict(mat_nuclides=_set(0, 3)),
    "nuclide_negative": dict(mat_nuclides=_set(1, -1)),
    "offset_start": dict(grid_offsets=_set(0, 1)),
}


@pytest.mark.parametrize("name", sorted(BAD_TABLES))
def test_create_rejects_bad_tables(lib, name):
    st, msg, h = _create_status(_mutated(**BAD_TABLES[name]))
    assert st == xs.XS_ETABLE, (st, msg)
    assert msg
    assert not h.value


def test_create_rejects_structure(lib):
    t = _small()
    assert _create_status(t, n_channels=4)[0] == xs.XS_ETABLE
    assert _create_status(t, n_nuclides=0)[0] == xs.XS_ETABLE
    assert _create_status(t, n_materials=0)[0] == xs.XS_ETABLE
    assert _create_status(t, flags=32)[0] == xs.XS_EINVAL
    # FP32 record pairs need the FP32 records
    assert _create_status(t, flags=xs.XS_BUILD_FP32_PAIRS)[0] == xs.XS_EINVAL
    assert _create_status(t, flags=xs.XS_BUILD_FP32_PAIRS |
                          xs.XS_BUILD_HASH, bins=4)[0] == xs.XS_EINVAL
    assert _create_status(t, flags=xs.XS_BUILD_UNION_BY_MATERIAL)[0] == xs.XS_EINVAL
    assert _create_status(t, flags=xs.XS_BUILD_HASH, bins=0)[0] == xs.XS_EINVAL
    assert _create_status(t, flags=xs.XS_BUILD_HASH, bins=100001)[0] == xs.XS_EINVAL
    # a nuclide with a single grid point
    one = synth.Tables(np.array([0, 1, 3], np.int64), np.array([0.5, 0.1, 0.9]),
                       np.ones((3, 5)), np.array([0, 1], np.int32),
                       np.array([0], np.int32), np.array([1.0]))
    assert _create_status(one)[0] == xs.XS_ETABLE
    # an empty material and a repeated nuclide
    t2 = synth.Tables(t.grid_offsets, t.energy, t.xs, np.array([0, 0, 2], np.int32),
                      np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    assert _create_status(t2)[0] == xs.XS_ETABLE
    t3 = synth.Tables(t.grid_offsets, t.energy, t.xs, np.array([0, 2], np.int32),
                      np.array([1, 1], np.int32), np.array([1.0, 1.0]))
    assert _create_status(t3)[0] == xs.XS_ETABLE


FP32_RANGE = {
    "xs_overflows_fp32": dict(xs=_set(4, 3.5e38)),
    "xs_subnormal_in_fp32": dict(xs=_set(6, 1e-39)),
    "xs_rounds_to_zero_in_fp32": dict(xs=_set(2, 1e-50)),
    "density_subnormal_in_fp32": dict(mat_density=_set(0, 1e-40)),
    "density_overflows_fp32": dict(mat_density=_set(1, 1e39)),
}


@pytest.mark.parametrize("name", sorted(FP32_RANGE))
def test_fp32_build_rejects_values_outside_fp32(lib, name):
    """Values that FP32 cannot hold as normal numbers are refused when the
    FP32 records are built, and accepted when they are not."""
    t = _mutated(**FP32_RANGE[name])
    st, msg, h = _create_status(t, xs.XS_BUILD_FP32)
    assert st == xs.XS_ETABLE and "FP32" in msg, (st, msg)
    assert not h.value
    st, msg, _ = _create_status(t, 0)
    assert st != xs.XS_ETABLE, msg  # FP64 tables hold them


def test_fp32_build_accepts_zero_and_the_normal_range(lib):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present; covered by the GPU tests")
    t = _mutated(xs=lambda a: a.reshape(-1).__setitem__(
        slice(0, 3), [0.0, np.finfo(np.float32).tiny, 3.0e38]))
    st, msg, _ = _create_status(t, xs.XS_BUILD_FP32)
    assert st == xs.XS_EHIP, (st, msg)  # past every host check


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.xs_create_tables(None, None, ctypes.byref(h)) == xs.XS_EINVAL
    assert lib.xs_destroy_tables(None) == xs.XS_OK
    assert lib.xs_lookup_batch(None, 10, None, None, None, None, None, 0,
                               None) == xs.XS_EINVAL
    assert lib.xs_lookup_indices(None, 1, None, None, None, None, 0,
                                 None) == xs.XS_EINVAL
    info = xs.xs_table_info_t()
    assert lib.xs_table_info(None, ctypes.byref(info)) == xs.XS_EINVAL
    assert lib.xs_profile_begin(None) == xs.XS_EINVAL


def test_valid_tables_pass_validation(lib):
    """A valid description gets past every host check; without a device the
    first HIP call is what fails."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present; covered by the GPU tests")
    st, msg, h = _create_status(_small(), xs.XS_BUILD_FP32 | xs.XS_BUILD_HASH, 100)
    assert st == xs.XS_EHIP, (st, msg)
