"""The C ABI library loads and exports every entry point the public headers declare.

No compute call is made (no GPU is needed): only host-side argument checking.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for f in os.listdir(INCLUDE):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(lm_[a-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2208_02682_amd.lagmean import LIB_PATH, load_library
    if not os.path.exists(LIB_PATH):
        # a fresh checkout: build it (hipcc cross-compiles for gfx950 without a GPU)
        from paper_2208_02682_amd.build import build
        build(verbose=False)
    return load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("lm_create", "lm_set_state", "lm_step", "lm_begin_interval", "lm_end_interval",
              "lm_read_mean", "lm_destroy", "lm_query_footprint"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_checks_without_a_gpu(lib):
    from paper_2208_02682_amd import LagMeanError, footprint, make_config
    # footprint is host-only and allocates nothing
    b64 = footprint(make_config(64, dt=0.01))
    b1k = footprint(make_config(1024, precision="fp32", dt=6e-4))
    assert 0 < b64 < b1k < 512 * 2**20
    for bad in (dict(n=100), dict(n=64, dt=0.0), dict(n=64, nu8=-1.0)):
        kw = dict(dt=0.01)
        kw.update(bad)
        n = kw.pop("n")
        with pytest.raises(LagMeanError):
            footprint(make_config(n, **kw))
    cfg = make_config(64, dt=0.01)
    cfg.mode = 7
    with pytest.raises(LagMeanError) as e:
        footprint(cfg)
    assert e.value.status == -6
    assert lib.lm_status_str(-5) == b"non-finite values in the outputs"
    # null handles are rejected, not dereferenced
    assert lib.lm_step(None, 1) == -1
    assert lib.lm_destroy(None) == 0


def test_product_path_does_not_import_the_oracle():
    import subprocess
    import sys
    code = ("import sys; import paper_2208_02682_amd, paper_2208_02682_amd.lagmean, paper_2208_02682_amd.build;"
            "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), 'oracle imported'")
    subprocess.run([sys.executable, "-c", code], check=True, cwd=ROOT)


def test_header_is_plain_c(tmp_path):
    # the boundary is a C ABI: the header compiles as C99 with warnings as errors
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "h.c"
    src.write_text('#include "lagmean.h"\nint main(void) { lm_schedule s = {0, 1, 1}; lm_config c; (void)s; (void)c;'
                   ' return (int)LM_OK; }\n')
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", INCLUDE, "-c", str(src), "-o",
                    str(tmp_path / "h.o")], check=True)
