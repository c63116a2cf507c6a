"""The C-ABI library loads, exports every entry point declared in
include/pm.h, and rejects bad configurations before touching a device."""
import os
import re

import pytest

from paper_2007_13394_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2007_13394_amd import pm
    lib = ctypes.CDLL(pm._SO)
    names = _declared()
    assert "pm_step" in names and "pm_init" in names and len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pm.EXPORTS) == names


def test_sizes_match_configuration_counts():
    from paper_2007_13394_amd import pm
    for name in ("C1", "C2", "C3", "C5"):
        c = I.config(name)
        P, nseg, nbytes = pm.pm_sizes(pm.make_config(c))
        nc, nn, _ = I.counts(c)
        assert P == nc + nn and nseg == 11
        n = c["n_mesh"]
        assert nbytes >= 8 * n ** 3 + 3 * n * n * (n // 2 + 1) * 8
    P, nseg, _ = pm.pm_sizes(pm.make_config(I.config("C1", n_sites=0)))
    assert P == 32 ** 3 and nseg == 1


@pytest.mark.parametrize("field,value", [("n_mesh", 48), ("n_mesh", 4096), ("n_cdm", 128), ("n_sites", 3),
                                         ("shift", 60), ("a0", 0.001), ("n_shell", 0), ("omega_m", 0.0)])
def test_bad_configuration_is_an_argument_error(field, value):
    from paper_2007_13394_amd import pm
    c = I.config("C1")
    c[field] = value
    with pytest.raises(pm.PMError) as e:
        pm.pm_sizes(pm.make_config(c))
    assert e.value.status == pm.PM_ERR_ARG


def test_init_rejects_null_workspace_without_device_work():
    import ctypes as C
    from paper_2007_13394_amd import pm
    cfg = pm.make_config(I.config("C1"))
    h = C.c_void_p()
    st = pm._lib.pm_init(C.byref(cfg), None, 0, None, C.byref(h))
    assert st == pm.PM_ERR_ARG and h.value is None
    st = pm._lib.pm_init(C.byref(cfg), C.c_void_p(256), 10, None, C.byref(h))
    assert st == pm.PM_ERR_SIZE
