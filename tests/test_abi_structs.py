"""The ctypes mirrors of the ABI structs have the C layout (sizes and field
offsets from the header, checked by compiling a probe with the host
compiler)."""
import ctypes as C
import os
import subprocess
import tempfile

from paper_1502_02935_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_struct_layouts_match_header():
    fields = {"mhd_config": L.mhd_config, "mhd_diag_t": L.mhd_diag_t,
              "mhd_profile_t": L.mhd_profile_t, "mhd_gate": L.mhd_gate}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mhd.h"', "int main(void) {"]
    for name, cls in fields.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().split("\n"))
    for name, cls in fields.items():
        assert int(got["%s size" % name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(got["%s.%s" % (name, f[0])]) == getattr(cls, f[0]).offset, (name, f[0])


def test_oracle_struct_layouts_match_header():
    from oracle import pyorc as O
    fields = {"orc_config": O._Cfg, "orc_diag": O._Diag}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "orc.h"', "int main(void) {"]
    for name, cls in fields.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "oracle"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().split("\n"))
    for name, cls in fields.items():
        assert int(got["%s size" % name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(got["%s.%s" % (name, f[0])]) == getattr(cls, f[0]).offset, (name, f[0])
