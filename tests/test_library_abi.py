"""CPU checks of the C ABI: the library builds, loads, exports what
include/sdc.h declares, validates its arguments, and generates network code
whose sparsity pattern matches a symbolic LU done here independently."""
import ctypes
import os
import re

import numpy as np
import pytest

import sdc_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdc.h")


@pytest.fixture(scope="module")
def binding():
    from paper_1910_12578_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libsdc.so not built: run __graft_entry__.build()")
    _binding.lib()
    return _binding


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(sdc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sdc_init", "sdc_advective_term", "sdc_reaction_solve", "sdc_sweep", "sdc_step",
                 "sdc_destroy", "sdc_last_error", "sdc_stats"):
        assert must in names


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol(binding):
    assert sorted(binding.EXPORTS) == declared_functions()


def test_config_struct_layout_matches_header(binding):
    # field order and count of sdc_config / sdc_network / sdc_nodes in the header
    text = open(HEADER).read()
    body = text[text.find("typedef struct {\n  int32_t dim;"):text.find("} sdc_config;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(\w+)(?:\[\d\])?;", body)
    assert [f[0] for f in binding.Config._fields_] == fields
    c = binding.Config()
    binding.lib().sdc_config_default(ctypes.byref(c))
    assert c.n_nodes == 3 and c.n_iters == 4 and c.newton_tol == 1e-13 and c.gamma == 1.4


@pytest.mark.parametrize("bad", [dict(dim=4), dict(n_nodes=6), dict(n_iters=0), dict(precision=3),
                                 dict(gamma=1.0), dict(newton_tol=0.0), dict(n=(1, 8))])
def test_invalid_configuration_is_rejected_without_a_gpu(binding, bad):
    net = si.random_network(7, 10, 202)
    cfg = dict(dim=2, n=(8, 8), dx=(0.1, 0.1))
    cfg.update(bad)
    c = binding.make_config(cfg)
    n, keep = binding.make_network(net)
    rc = binding.lib().sdc_generated_source(ctypes.byref(c), ctypes.byref(n), None, 0)
    assert rc < 0
    assert binding.lib().sdc_last_error(None)


def test_invalid_network_is_rejected(binding):
    net = si.random_network(7, 10, 202)
    net = dict(net, reactants=net["reactants"].copy())
    net["reactants"][3, 0] = 9
    with pytest.raises(binding.SDCError) as e:
        binding.generated_source(dict(dim=1, n=(8,), dx=(0.1,)), net)
    assert "reactant" in str(e.value)


def _symbolic_lu_nnz(net):
    """Structural nonzeros of I - dt dR/dx and of its LU in index order."""
    ns = net["nspec"]
    n = ns + 1
    P = np.eye(n, dtype=bool)
    for r in range(net["nreact"]):
        cols = [c for c in net["reactants"][r] if c >= 0] + [ns]
        rows = list(np.nonzero(net["stoich"][r])[0]) + [ns]
        for i in rows:
            for j in cols:
                P[i, j] = True
    nj = int(P.sum())
    fma = 0
    for k in range(n):
        for i in range(k + 1, n):
            if P[i, k]:
                for j in range(k + 1, n):
                    if P[k, j]:
                        P[i, j] = True
                        fma += 1
    return nj, int(P.sum()), fma


@pytest.mark.parametrize("name,net", [("chain", si.chain_network()),
                                      ("net7", si.random_network(7, 10, 202)),
                                      ("net13", si.random_network(13, 20, 302))])
def test_generated_pattern_matches_symbolic_lu(binding, name, net):
    src = binding.generated_source(dict(dim=1, n=(8,), dx=(0.1,)), net)
    m = re.search(r"Newton matrix: (\d+) structural nonzeros, (\d+) with LU fill-in, (\d+) factorisation", src)
    assert m, src[:400]
    assert tuple(int(v) for v in m.groups()) == _symbolic_lu_nnz(net)
    assert f"#define SDC_NS {net['nspec']}" in src
    # no packed FP32 math requested anywhere, kernels present
    for k in ("sdc_advect", "sdc_transition_first", "sdc_transition_node0", "sdc_transition_later",
              "sdc_reaction_solve", "sdc_source"):
        assert k in src


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1910_12578_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h", ".hpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_ahead_of_time_kernels_of_the_standard_workloads(binding):
    """build() compiles the standard workloads' kernels with hipcc into the
    kernel cache under the name the runtime looks for first."""
    names = set()
    for name, shape in (("net2d", (8, 8)), ("net3d", (4, 4, 4))):
        w = si.workload(name, shape=shape)
        for prec in (0, 1):
            path = binding.aot_name(binding.config_from_workload(w, precision=prec), w["network"])
            assert path == binding.aot_name(binding.config_from_workload(w, precision=prec), w["network"])
            assert path.endswith(".aot.co") and os.path.basename(os.path.dirname(path)) == "_kcache"
            assert os.path.getsize(path) > 0, path
            names.add(path)
    assert len(names) == 4
