"""C-ABI checks that need no GPU: the library loads and exports every
function include/thor.h declares; the binding mirrors the struct layouts."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2507_11603_amd import thor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(thor_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(thor.LIB_PATH):
        pytest.fail("libthor.so not built; run __graft_entry__.build()")
    return thor.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(thor.SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", thor.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(r"\bT %s$" % n, out, flags=re.M), n


def test_struct_layouts_match_header():
    """Compile a tiny host program against thor.h printing sizeof/offsetof and
    compare with the ctypes mirrors."""
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "thor_rays.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(thor_geometry), sizeof(thor_source),
         sizeof(thor_transport_opts), sizeof(thor_stats), sizeof(thor_record),
         sizeof(thor_shell_request));
  printf("%zu %zu %zu %zu\n", offsetof(thor_geometry, n_HI_field), offsetof(thor_geometry, g_hg),
         offsetof(thor_transport_opts, step_events), offsetof(thor_transport_opts, records));
  printf("%zu %zu %zu %zu %zu\n", sizeof(thor_ray_grid), sizeof(thor_forest_opts),
         offsetof(thor_ray_grid, ds), offsetof(thor_forest_opts, u_lo),
         offsetof(thor_forest_opts, precision));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "t.c")
        open(p, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, p])
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = list(map(int, lines[0].split()))
    offs = list(map(int, lines[1].split()))
    assert sizes == [C.sizeof(thor.thor_geometry), C.sizeof(thor.thor_source),
                     C.sizeof(thor.thor_transport_opts), C.sizeof(thor.thor_stats),
                     C.sizeof(thor.thor_record), C.sizeof(thor.thor_shell_request)]
    assert offs == [thor.thor_geometry.n_HI_field.offset, thor.thor_geometry.g_hg.offset,
                    thor.thor_transport_opts.step_events.offset, thor.thor_transport_opts.records.offset]
    assert thor.RECORD_DTYPE.itemsize == C.sizeof(thor.thor_record)
    rays = list(map(int, lines[2].split()))
    assert rays == [C.sizeof(thor.thor_ray_grid), C.sizeof(thor.thor_forest_opts),
                    thor.thor_ray_grid.ds.offset, thor.thor_forest_opts.u_lo.offset,
                    thor.thor_forest_opts.precision.offset]


def test_create_without_device_fails_cleanly(lib):
    """No GPU here: thor_create must return an error code, not crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = C.c_void_p()
    code = lib.thor_create(C.byref(h), 0, None, 0)
    assert code < 0 and not h.value
    assert lib.thor_last_error()


def test_ray_calls_validate_on_the_host(lib):
    """Invalid raytracing arguments are refused before any device work, with
    a message; a call with no rays is a no-op (no GPU needed for either)."""
    g = thor.thor_ray_grid(4, 4, 4, 3, 1.0)
    assert lib.thor_ray_project(C.byref(g), None, None, None, None, None) == -1
    assert b"axis" in lib.thor_ray_last_error()
    g.axis, g.ds = 2, -1.0
    assert lib.thor_ray_project(C.byref(g), None, None, None, None, None) == -1
    g.ds = 1.0
    o = thor.thor_forest_opts(0, 5, 0, 1, 0.0, 1, 8, 0.0, 1.0, 0)
    assert lib.thor_ray_forest(C.byref(g), C.byref(o), None, None, None, None, None) == -1
    assert b"outside" in lib.thor_ray_last_error()
    o.ni, o.n_sub = 4, 0
    assert lib.thor_ray_forest(C.byref(g), C.byref(o), None, None, None, None, None) == -1
    o.n_sub, o.nb = 1, (1 << 22) + 1
    assert lib.thor_ray_forest(C.byref(g), C.byref(o), None, None, None, None, None) == -1
    o.nb, o.u_hi = 8, 0.0
    assert lib.thor_ray_forest(C.byref(g), C.byref(o), None, None, None, None, None) == -1
    o.u_hi, o.precision = 1.0, 7
    assert lib.thor_ray_forest(C.byref(g), C.byref(o), None, None, None, None, None) == -1
    o.precision, o.nj = 0, 0
    assert lib.thor_ray_forest(C.byref(g), C.byref(o), None, None, None, None, None) == 0


def test_ray_outputs_are_checked_before_any_call():
    """A caller-supplied output of the wrong shape, dtype or layout is refused
    before the library writes into it (the check needs no GPU)."""
    import torch
    dev = torch.device("cpu")
    ok = torch.zeros((4, 3), dtype=torch.float64)
    assert thor._check_out(ok, "out", (4, 3), dev) is ok
    for bad in (torch.zeros((3, 4), dtype=torch.float64), torch.zeros((4, 3), dtype=torch.float32),
                torch.zeros((3, 4), dtype=torch.float64).t(), "not a tensor"):
        with pytest.raises(ValueError):
            thor._check_out(bad, "out", (4, 3), dev)
