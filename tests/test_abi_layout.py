"""CPU: the binding's ctypes structures have the fields of include/usp.h's
structs, in the same order and with the same sizes, so that a field added
on one side only (a new numerics switch, say) fails here rather than
shifting every later field the library reads; the same for the oracle's
configuration record and its binding."""
import ctypes as C
import os
import re

import pytest

from paper_1808_03801_amd import usp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_SIZES = {"double": 8, "int": 4, "uint64_t": 8, "long long": 8, "size_t": 8,
           "uint32_t": 4, "int32_t": 4}


def _c_structs(header=os.path.join("include", "usp.h")):
    """name -> [(field, bytes)] of every `typedef struct { ... } name;`"""
    text = open(os.path.join(ROOT, header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    out = {}
    sizes = dict(C_SIZES)
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in (d.strip() for d in body.split(";")):
            if not decl:
                continue
            m = re.match(r".*\(\s*\*\s*(\w+)\s*\)\s*\(.*\)$", decl, flags=re.S)
            if m:  # function pointer
                fields.append((m.group(1), 8))
                continue
            m = re.match(r"((?:const\s+)?(?:long long|unsigned\s+\w+|\w+)\s*\**)\s*(.*)$", decl,
                         flags=re.S)
            ctype, rest = m.group(1).strip(), m.group(2)
            for d in rest.split(","):
                d = d.strip()
                ptr = d.startswith("*") or ctype.endswith("*")
                dm = re.match(r"\**\s*(\w+)\s*(?:\[(\d+)\])?$", d)
                fname, n = dm.group(1), int(dm.group(2) or 1)
                base = re.sub(r"^const\s+", "", ctype).rstrip("* ").strip()
                if ptr:
                    fields.append((fname, 8 * n))
                elif sizes.get(base) is None:
                    # a struct declared earlier in the header: sized by the
                    # binding's type of the same field (checked on its own)
                    fields.append((fname, None))
                else:
                    fields.append((fname, sizes[base] * n))
        out[name] = fields
        sizes[name] = None
    return out


PAIRS = [("usp_gas", usp.Gas), ("usp_face", usp.Face), ("usp_problem", usp.ProblemC),
         ("usp_numerics", usp.Numerics), ("usp_device", usp.Device),
         ("usp_moments_view", usp.MomentsView), ("usp_stats_t", usp.Stats)]


@pytest.mark.parametrize("cname,ctype", PAIRS, ids=[p[0] for p in PAIRS])
def test_ctypes_struct_matches_header(cname, ctype):
    cf = _c_structs()[cname]
    pf = [(f[0], C.sizeof(f[1])) for f in ctype._fields_]
    # a nested struct field (usp_face face[4]) is sized by its ctypes type
    cf = [(n, dict(pf).get(n) if b is None else b) for n, b in cf]
    assert [n for n, _ in cf] == [n for n, _ in pf], (cname, cf, pf)
    assert cf == pf, (cname, cf, pf)


def test_oracle_config_matches_its_header():
    from oracle import oracle as O
    cf = _c_structs(os.path.join("oracle", "usp_oracle.h"))["uspo_config"]
    pf = [(f[0], C.sizeof(f[1])) for f in O.Config._fields_]
    assert cf == pf, (cf, pf)


def test_footprint_counts_the_particle_buffers():
    """usp_footprint (host arithmetic, no device): the two particle buffers
    of (dim + 4) components per slot dominate, and the figure grows with the
    cells, the capacity and the state precision"""
    from paper_1808_03801_amd import problems as P
    if not os.path.exists(usp.LIB_PATH):
        pytest.skip("libusp.so not built")
    pb = P.cavity_2d(Kn=0.01, n=32, ppc=100, seed=1)
    cap = (pb.max_ppc + 63) // 64 * 64
    parts = 2 * (pb.dim + 4) * pb.ncell * cap * 4
    f = usp.footprint(pb)
    assert parts <= f <= 1.5 * parts
    assert usp.footprint(pb.replace(precision=64)) > 1.9 * parts
    assert usp.footprint(pb.replace(max_ppc=2 * pb.max_ppc)) > 1.9 * parts
    assert usp.footprint(P.cavity_2d(Kn=0.01, n=64, ppc=100, seed=1)) > 3.9 * parts
