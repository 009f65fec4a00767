"""CPU checks of the C ABI: the built library loads and exports every function
declared in include/lb_chiral.h and include/lb_nematic2d.h, and the Python
binding declares the same set.  No compute call is made (there may be no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb_chiral.h")
HEADER_2D = os.path.join(ROOT, "include", "lb_nematic2d.h")


def declared_functions(header=HEADER, prefix="lb_"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for n in ("lb_init", "lb_step", "lb_moments", "lb_free_energy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2011_00287_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("library not built: run python -m paper_2011_00287_amd.build")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared_functions() + declared_functions(HEADER_2D, "lb2d_"):
        assert hasattr(L, n), n


def test_binding_matches_header():
    from paper_2011_00287_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()
    assert sorted(_lib.SIGNATURES_2D) == declared_functions(HEADER_2D, "lb2d_")


def _struct_fields(header, name):
    text = open(header).read()
    body = re.search(r"typedef struct \{([^}]*)\} " + name + ";", text).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for n in decl.split(None, 1)[1].split(","):
            fields.append(re.sub(r"\[.*\]", "", n).strip())
    return fields


def test_2d_struct_layouts():
    from paper_2011_00287_amd import _lib
    assert _struct_fields(HEADER_2D, "lb2d_params") == [f[0] for f in _lib.Lb2dParams._fields_]
    assert _struct_fields(HEADER_2D, "lb2d_totals") == [f[0] for f in _lib.Lb2dTotals._fields_]


def test_2d_invalid_params_rejected_on_the_host():
    import numpy as np
    from paper_2011_00287_amd import _lib, sim2d
    p = dict(tau=2.5, rho0=1.0, A0=0.1, chi=4.0, K=0.04, Gamma=0.3, xi=0.7, zeta=0.0)
    for bad, q2 in ((dict(p, tau=0.5), np.zeros((2, 4, 4))), (p, np.zeros((2, 2, 4))),
                    (dict(p, K=float("inf")), np.zeros((2, 4, 4)))):
        with pytest.raises(_lib.LbError) as e:
            sim2d.Nematic2D(bad, q2)
        assert e.value.status == _lib.LB_EINVAL
    with pytest.raises(_lib.LbError) as e:
        sim2d.Nematic2D(p, np.zeros((2, 4, 4)), precision="fp16s")
    assert e.value.status == _lib.LB_EINVAL


def test_param_struct_layout():
    """Field order of lb_params in the header equals the ctypes struct."""
    from paper_2011_00287_amd import _lib
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} lb_params;", text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1]
        for n in names.split(","):
            fields.append(re.sub(r"\[.*\]", "", n).strip())
    assert fields == [f[0] for f in _lib.LbParams._fields_]


def test_last_error_is_empty_string_initially():
    from paper_2011_00287_amd import _lib
    assert _lib.lib().lb_last_error() in (b"",)


def test_destroy_is_null_safe():
    from paper_2011_00287_amd import _lib
    _lib.lib().lb_destroy(None)


def test_invalid_params_rejected_before_any_device_work():
    """Validation runs on the host: a bad tau fails with LB_EINVAL even without a GPU."""
    import numpy as np
    from paper_2011_00287_amd import _lib, inputs, sim
    p = dict(inputs.BASE_PARAMS, tau=0.4)
    phi = np.zeros((4, 4, 4))
    q5 = np.zeros((5, 4, 4, 4))
    with pytest.raises(_lib.LbError) as e:
        sim.Sim(p, phi, q5)
    assert e.value.status == _lib.LB_EINVAL
    p = dict(inputs.BASE_PARAMS)
    with pytest.raises(_lib.LbError) as e:
        sim.Sim(p, np.zeros((2, 4, 4)), np.zeros((5, 2, 4, 4)))
    assert e.value.status == _lib.LB_EINVAL
    with pytest.raises(_lib.LbError) as e:
        sim.Sim(dict(p, zeta=float("nan")), phi, q5)
    assert e.value.status == _lib.LB_EINVAL


def test_oversize_box_rejected_before_allocation():
    """A box above 2^29 sites is refused with LB_ENOMEM during validation."""
    import numpy as np
    from paper_2011_00287_amd import _lib, inputs, sim
    p = dict(inputs.BASE_PARAMS)
    lp = sim.make_params(p, (1024, 1024, 1024), "fp32")
    import ctypes
    h = ctypes.c_void_p()
    phi = np.zeros(1)
    q5 = np.zeros(5)
    st = _lib.lib().lb_init(ctypes.byref(lp), phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            q5.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None, ctypes.byref(h))
    assert st == _lib.LB_ENOMEM
    assert not h.value


def test_header_is_plain_c_and_links():
    """A C11 program using only include/lb_chiral.h compiles without warnings
    and links against the built library (it runs in the GPU tests)."""
    import tempfile
    from c_abi_build import compile_c_consumer
    from paper_2011_00287_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("library not built: run python -m paper_2011_00287_amd.build")
    with tempfile.TemporaryDirectory() as d:
        exe = compile_c_consumer(d)
        assert os.path.exists(exe)


def test_tuning_struct_layout():
    """Field order of lb_tuning in the header equals the ctypes struct."""
    from paper_2011_00287_amd import _lib
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{([^{}]*)\} lb_tuning;", text).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = [d.strip().split(None, 1)[1].strip() for d in body.split(";") if d.strip()]
    assert fields == [f[0] for f in _lib.LbTuning._fields_]


@pytest.mark.parametrize("bad", [{"path": 4}, {"path": -1}, {"lb_tile": 6}, {"order_tile": -1}, {"pc_tile": 5},
                                 {"pcmu_tile": 9}, {"step_tile": 4}, {"adj_tile": 3}, {"adj_order_tile": 3},
                                 {"tz_step": -1}, {"tz_adj": -2}])
def test_invalid_tuning_rejected_before_any_device_work(bad):
    """lb_init_tuned validates the launch configuration on the host (LB_EINVAL)."""
    import numpy as np
    from paper_2011_00287_amd import _lib, inputs, sim
    phi = np.zeros((4, 4, 4))
    q5 = np.zeros((5, 4, 4, 4))
    with pytest.raises(_lib.LbError) as e:
        sim.Sim(dict(inputs.BASE_PARAMS), phi, q5, tuning=bad)
    assert e.value.status == _lib.LB_EINVAL


def test_one_launch_path_refused_with_the_pc4_integrator():
    import numpy as np
    from paper_2011_00287_amd import _lib, inputs, sim
    phi = np.zeros((4, 4, 4))
    q5 = np.zeros((5, 4, 4, 4))
    with pytest.raises(_lib.LbError) as e:
        sim.Sim(dict(inputs.BASE_PARAMS), phi, q5, fd_scheme="pc4", tuning={"path": "one"})
    assert e.value.status == _lib.LB_EINVAL
    with pytest.raises(KeyError):
        sim.make_tuning({"no_such_field": 1})


def test_centre_noalloc_rejects_bad_arguments_before_any_device_work():
    """Sizes, precision and pointers are checked on the host (no GPU is touched)."""
    from paper_2011_00287_amd import _lib
    L = _lib.lib()
    assert L.lb_centre_noalloc(1024, 1024, 33, _lib.LB_FP64, 16, 16, None) == _lib.LB_EINVAL
    assert L.lb_centre_noalloc(0, 4, 4, _lib.LB_FP64, 16, 16, None) == _lib.LB_EINVAL
    assert L.lb_centre_noalloc(4, 4, 4, 7, 16, 16, None) == _lib.LB_EINVAL
    assert L.lb_centre_noalloc(4, 4, 4, _lib.LB_FP32, None, 16, None) == _lib.LB_EINVAL


def test_kernel_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    """The counter records are valid for the kernel code they were taken on: an
    edited comment or blank line keeps the hash, an edited statement changes it."""
    import shutil

    from paper_2011_00287_amd import build

    base = build.kernel_source_hash()
    csrc = tmp_path / "csrc"
    shutil.copytree(os.path.join(build.PKG, "csrc"), csrc)
    monkeypatch.setattr(build, "PKG", str(tmp_path))
    assert build.kernel_source_hash() == base
    f = csrc / "kernels_fused.hpp"
    text = f.read_text()
    f.write_text("// an added comment\n\n" + text.replace("namespace lbc {", "namespace lbc {  /* note */", 1))
    assert build.kernel_source_hash() == base
    f.write_text(text.replace("R(0.5)", "R(0.25)", 1))
    assert build.kernel_source_hash() != base
