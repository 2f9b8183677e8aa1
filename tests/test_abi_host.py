"""The C ABI on the CPU (no GPU needed): the library loads and exports every
function include/bddc.h declares; a host-only context (device < 0) runs the
setup analysis, whose results equal the oracle's -- glob and corner counts,
the constraint count Nc, every substructure matrix A_i (Sec. 2: subassembled
from element matrices) with its local dof numbering, and the weights of the
averaging operator E (Sec. 7: diagonal entries of the substructure matrices);
and calls out of order or with bad arguments return their documented status.
No compute call is made."""
import os
import re

import numpy as np
import pytest

import meshgen
from paper_0910_5863_amd import BDDC, BddcError, binding, load

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "bddc.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bddc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = load()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(binding.SYMBOLS)


CASES = {
    "poisson16": (lambda: meshgen.poisson_16(), "ce"),
    "elast6x3_cef": (lambda: meshgen.small_elasticity_layers(6, 3, contrast=1e3), "cef"),
    "kmeans_elast": (lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3), "ce"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_analysis_matches_oracle(name):
    from oracle.fem import Substructures
    from oracle.interface import Interface
    from oracle.cov import Constraints
    make, mode = CASES[name]
    p = make()
    S = Substructures(p)
    itf = Interface(S)
    cons = Constraints(itf, mode)
    b = BDDC(device=-1)
    b.setup(p, mode)
    info = b.info()
    c = itf.counts()
    assert info.n_glob == p.n_glob == S.n_glob
    assert info.n_sub == p.n_sub
    assert (info.n_corners, info.n_edges, info.n_faces) == (c["corners"], c["edges"], c["faces"])
    assert info.nc == cons.Nc()
    for s in range(p.n_sub):
        gdof, n_int, A, w = b.substructure(s)
        # local order: interior dofs first, then interface dofs, each ascending
        g = S.gdof[s]
        interior, iface = g[itf.interior[s]], g[itf.iface[s]]
        assert n_int == interior.size
        assert np.array_equal(gdof, np.concatenate([np.sort(interior), np.sort(iface)]))
        # same matrix up to the local permutation
        loc = {int(v): k for k, v in enumerate(g)}
        perm = np.array([loc[int(v)] for v in gdof])
        Ao = S.A[s][perm][:, perm].toarray()
        scale = np.abs(Ao).max()
        assert np.abs(A.toarray() - Ao).max() <= 1e-14 * scale
        # weights of E on the interface dofs
        dl = itf.delta[s][perm[n_int:]]
        assert np.allclose(w, dl, rtol=1e-14, atol=0)
    b.close()


def test_host_only_context_rejects_device_calls():
    p = meshgen.poisson_16()
    b = BDDC(device=-1)
    with pytest.raises(BddcError) as e:
        b.factor()
    assert e.value.code == 2          # BDDC_ERR_STATE: before setup
    b.setup(p, "ce")
    for call in (b.factor, lambda: b.adapt(10.0)):
        with pytest.raises(BddcError) as e:
            call()
        assert e.value.code == 2      # host-only context
    with pytest.raises(BddcError) as e:
        b.substructure(p.n_sub)       # no such substructure
    assert e.value.code == 1          # BDDC_ERR_ARG
    b.close()


def test_bad_setup_arguments():
    p = meshgen.poisson_16()
    b = BDDC(device=-1)
    bad = meshgen.poisson_16()
    bad.elem_sub = bad.elem_sub.copy()
    bad.elem_sub[0] = p.n_sub          # out of range
    with pytest.raises(BddcError) as e:
        b.setup(bad, "ce")
    assert e.value.code == 1
    b.close()


def test_insufficient_corners_rejected_without_augmentation():
    """Assumption 2 (Sec. 3): without the corner augmentation, a k-means
    partition whose face pairs see fewer than three non-collinear corners is
    rejected by bddc_setup with BDDC_ERR_INSUFFICIENT_CORNERS; the same
    partition with augmentation, and a cube partition without it, are
    accepted."""
    # 10^3 elements in 6 k-means parts: two floating face pairs lack corners
    km = meshgen.small_kmeans(meshgen.ELASTICITY, 10, 6, contrast=1e3)
    b = BDDC(device=-1)
    with pytest.raises(BddcError) as e:
        b.setup(km, "ce", augment_corners=False)
    assert e.value.code == 7
    assert "Assumption 2" in str(e.value)
    b.close()
    b = BDDC(device=-1)
    b.setup(km, "ce", augment_corners=True)
    b.close()
    b = BDDC(device=-1)
    b.setup(meshgen.small_elasticity_layers(6, 2, contrast=1e3), "ce", augment_corners=False)
    b.close()


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding that the header defines has the
    header's size and field offsets (gcc compiles the header as C and prints
    them)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    txt = open(HEADER).read()
    structs = [v for k, v in vars(binding).items()
               if isinstance(v, type) and issubclass(v, ctypes.Structure)
               and re.search(r"}\s*%s\s*;" % k, txt)]
    assert len(structs) >= 5
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bddc.h"', "int main(void) {"]
    expect = []
    for st in structs:
        lines.append('printf("%%zu\\n", sizeof(%s));' % st.__name__)
        expect.append(ctypes.sizeof(st))
        for name, *_ in st._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (st.__name__, name))
            expect.append(getattr(st, name).offset)
    lines.append("return 0; }")
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == expect


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so,
    before touching any device."""
    import subprocess
    import sys
    root = os.path.join(os.path.dirname(__file__), "..")
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
