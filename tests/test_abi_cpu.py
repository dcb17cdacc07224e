"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol that include/pbmp.h declares, the binding's structures match
the header's field lists, and defaults are those documented."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbmp.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1810_03698_amd import pbmp
    if not os.path.exists(pbmp.LIB_PATH):
        from paper_1810_03698_amd import build
        build.build()
    return pbmp.load()


def _declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pbmp_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def _struct_fields(name):
    txt = open(HEADER).read()
    m = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), txt, re.S)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        parts = decl.replace("*", " ").split()
        for f in " ".join(parts[1:]).split(","):
            fields.append(re.sub(r"\[\d+\]$", "", f.strip()))
    return fields


def test_binding_structs_match_header():
    from paper_1810_03698_amd import pbmp
    assert [f for f, _ in pbmp.Options._fields_] == _struct_fields("pbmp_options")
    assert [f for f, _ in pbmp.Result._fields_] == _struct_fields("pbmp_result")
    assert [f for f, _ in pbmp.KernelStats._fields_] == _struct_fields("pbmp_kstats")


def test_default_options(lib):
    from paper_1810_03698_amd import pbmp
    o = pbmp.Options()
    lib.pbmp_default_options(ctypes.byref(o))
    assert (o.eps_in, o.eps_out, o.kappa) == (1.0, 80.0, 0.125)
    assert (o.gauss_far, o.near_eta, o.mode) == (3, 2.0, 2)
    assert (o.theta, o.order_P, o.leaf_panels) == (0.5, 4, 300)
    assert (o.gmres_restart, o.gmres_tol) == (50, 1e-6)
    assert (o.scf_tol_debye, o.scf_omega, o.thole_a) == (1e-6, 0.7, 0.39)
    assert o.precision == 1 and o.hip_stream is None
    assert o.warm_start == 0 and o.verbose == 0


def test_product_path_has_no_oracle_dependency():
    """The package and the HIP sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1810_03698_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "bie_c" not in txt, f
