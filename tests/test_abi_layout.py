"""CPU check that the ctypes structures of the binding have the layout of
the structs declared in include/corutv.h: the same fields, in the same order,
at the same offsets, with the same total size (natural C alignment on
x86-64).  A field added on one side only would otherwise shift every later
field silently."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "corutv.h")

SCALARS = {"int32_t": 4, "uint32_t": 4, "int64_t": 8, "uint64_t": 8, "double": 8}
BINDING = {"corutv_mat": "Mat", "corutv_opts": "Opts", "corutv_info": "Info", "corutv_config": "Config",
           "corutv_rpca_info": "RpcaInfo", "corutv_request": "Request", "corutv_pass_stats": "PassStats"}


def header_structs():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for name, body in re.findall(r"typedef struct (\w+) \{(.*?)\}\s*\1\s*;", src, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            # "type a, b, c" declares several fields of one type
            m = re.match(r"(.*?)(\w+(?:\s*,\s*\w+)*)$", decl)
            ty = m.group(1).strip()
            for fname in m.group(2).split(","):
                fields.append((fname.strip(), ty))
        out[name] = fields
    return out


def layout(structs, name):
    """[(field, offset)], size, alignment of a header struct."""
    off, align, res = 0, 1, []
    for fname, ty in structs[name]:
        if "*" in ty:
            size = a = 8
        elif ty.replace("const ", "") in SCALARS:
            size = a = SCALARS[ty.replace("const ", "")]
        else:
            _, size, a = layout(structs, ty)
        off = (off + a - 1) // a * a
        res.append((fname, off))
        off += size
        align = max(align, a)
    return res, (off + align - 1) // align * align, align


def test_header_parses():
    s = header_structs()
    assert set(BINDING) <= set(s), sorted(s)


@pytest.mark.parametrize("cname", sorted(BINDING))
def test_binding_matches_header(cname):
    import paper_1906_04572_amd as cu

    structs = header_structs()
    fields, size, _ = layout(structs, cname)
    cls = getattr(cu, BINDING[cname])
    py = [(f, getattr(cls, f).offset) for f, _ in cls._fields_]
    assert [f for f, _ in py] == [f for f, _ in fields], (cname, py, fields)
    assert py == fields, (cname, py, fields)
    assert ctypes.sizeof(cls) == size, (cname, ctypes.sizeof(cls), size)
