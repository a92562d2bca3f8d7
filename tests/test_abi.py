"""Host-side checks of the C ABI: the library loads and exports every entry point
that include/hqa.h declares, and struct layouts of the binding match the header.
No compute call is made (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libhqa():
    from paper_2004_03972_amd import hqa
    if not os.path.exists(hqa._LIB_PATH):
        from paper_2004_03972_amd.csrc import build as b
        b.build()
    return hqa.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "hqa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hqa_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hqa_md_init", "hqa_md_run", "hqa_classify", "hqa_ising_energy"):
        assert n in names


def test_library_exports_every_declared_symbol(libhqa):
    for name in _declared():
        assert hasattr(libhqa, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2004_03972_amd import hqa
    assert sorted(hqa.EXPORTED) == _declared()
    for name in _declared():
        assert callable(getattr(hqa, name))


def test_abi_version_and_defaults(libhqa):
    from paper_2004_03972_amd import hqa
    assert hqa.hqa_abi_version() == hqa.ABI_VERSION == 10
    s = hqa.hqa_schedule_default()
    # Methods, "Scheduling functions for MD": (0.008, 4, 3), (0.12, 0.05, 1); M = 6 (Results)
    assert (s.alpha_f, s.rho1, s.rho2, s.beta_f, s.kappa1, s.kappa2) == (0.008, 4, 3, 0.12, 0.05, 1)
    assert s.M == 6 and s.W == 100 and s.r_g == 1.0
    o = hqa.hqa_md_opts_default()
    assert o.replicas == 1 and o.precision == hqa.HQA_PREC_F32 and o.plan == hqa.HQA_PLAN_AUTO


def test_struct_sizes_match_header():
    from paper_2004_03972_amd import hqa
    # sizes computed from the header's field lists under the x86-64 SysV ABI
    assert C.sizeof(hqa.hqa_problem) == 4 * 4 + 8 * 3 + 8 + 8
    assert C.sizeof(hqa.hqa_schedule) == 6 * 8 + 8 + 4 + 4 + 8 + 4 + 4 + 8
    assert C.sizeof(hqa.hqa_md_opts) == 4 + 4 + 8 + 8 + 8 + 4 * 4
    assert C.sizeof(hqa.hqa_classify_out) == 7 * 8


def test_invalid_arguments_rejected_before_device_work(libhqa):
    # argument checks that precede any HIP call
    from paper_2004_03972_amd import hqa
    import numpy as np
    J = np.zeros((4, 4))
    P = hqa.Problem(J)
    s = hqa.make_schedule(T=10, W=20)          # W > T
    o = hqa.hqa_md_opts_default()
    with pytest.raises(hqa.HQAError) as e:
        hqa.hqa_md_init([P.c], s, o)
    assert e.value.status == hqa.HQA_EINVAL
    s = hqa.make_schedule(T=10, W=5, M=5)      # odd M
    with pytest.raises(hqa.HQAError) as e:
        hqa.hqa_md_init([P.c], s, o)
    assert e.value.status == hqa.HQA_EINVAL
    s = hqa.make_schedule(T=10, W=5)
    o.precision = hqa.HQA_PREC_BF16
    rp, ci, v = np.array([0, 0, 0, 0, 0]), np.zeros(0), np.zeros(0)
    Pc = hqa.Problem(row_ptr=rp, col=ci, val=v)
    with pytest.raises(hqa.HQAError) as e:
        hqa.hqa_md_init([Pc.c], s, o)
    assert e.value.status == hqa.HQA_EUNSUPPORTED
    o.precision = hqa.HQA_PREC_F32
    o.flags = 2                                 # only HQA_MD_GRAPH is defined
    with pytest.raises(hqa.HQAError) as e:
        hqa.hqa_md_init([P.c], s, o)
    assert e.value.status == hqa.HQA_EINVAL and "flags" in str(e.value)


def test_classify_many_refuses_bad_arguments_on_the_host(libhqa):
    from paper_2004_03972_amd import hqa
    import numpy as np
    E = np.empty(4)
    with pytest.raises(hqa.HQAError) as e:
        hqa.hqa_classify_many(None, np.zeros(1, np.int32), 1, 2, 1, E, None, hqa.HQA_HOST)
    assert e.value.status == hqa.HQA_EINVAL and "handle" in str(e.value)


def test_pass_refuses_bad_arguments_on_the_host(libhqa):
    from paper_2004_03972_amd import hqa
    import numpy as np
    E = np.empty(4)
    with pytest.raises(hqa.HQAError) as e:
        hqa.hqa_md_pass(None, 1, 2, 1, E, None, hqa.HQA_MD_GRAPH)
    assert e.value.status == hqa.HQA_EINVAL and "handle" in str(e.value)
