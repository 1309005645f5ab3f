"""Host-side checks of the C ABI without a GPU: the library loads, exports
every symbol declared in include/ek.h, and the header's structs match the
binding's layout."""
import os
import re
import subprocess

import pytest

from paper_1607_04572_amd import ek as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    out = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            out += re.findall(r"^\s*(?:int|const char\*)\s+(ek_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(out))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(E.LIB_PATH):
        pytest.fail("libek_hip.so not built (run __graft_entry__.build())")
    names = subprocess.run(["nm", "-D", "--defined-only", E.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\w+)$", names, flags=re.M))
    decl = declared_symbols()
    assert decl, "no declarations found"
    missing = [s for s in decl if s not in exported]
    assert not missing, missing
    for s in decl:
        assert s in E.SYMBOLS or s.startswith("ek_batch"), s


def test_library_loads_and_reports_errors_without_gpu():
    L = E.lib()
    assert L.ek_strerror(0) == b"ok"
    assert b"size" in L.ek_strerror(-2)
    p = E.ek_params()
    p.nx, p.ny, p.nz = 10, 32, 32  # 10 = 2 * 5 is not 2^a 3^b
    p.agrid = p.tau = p.kT = p.fluid_density = 1.0
    p.viscosity = 1 / 6
    p.n_species = 1
    p.species[0].D = 0.3
    p.max_particles = 1
    with pytest.raises(E.EkError) as e:
        E.ek_query_footprint(p)
    assert e.value.code == -2
    p.nx = 32
    p.species[0].D = 0.4  # above the explicit-diffusion stability bound
    with pytest.raises(E.EkError) as e:
        E.ek_query_footprint(p)
    assert e.value.code == -3
    p.species[0].D = 0.39
    n = E.ek_query_footprint(p)
    assert n > 32 ** 3 * 19 * 8 * 2


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against include/ek.h with gcc and compare sizes and
    field offsets with the ctypes mirrors of the binding."""
    import ctypes as C
    structs = {"ek_species": E.ek_species, "ek_params": E.ek_params, "ek_particle": E.ek_particle,
               "ek_diag": E.ek_diag}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ek.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, val = line.split()
        cls = structs[name]
        got = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), (name, field, got, val)
