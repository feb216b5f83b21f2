"""The binding's ctypes structures against the C header (no GPU): the size of
every parameter and info struct and the offset of every field, as a program
compiled by the host C compiler against include/wcamg.h prints them.  A field
added, dropped, renamed or retyped on one side only fails here."""
import os
import shutil
import subprocess

import pytest

from paper_2111_05012_amd import wcamg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, 'include')

PAIRS = [(wcamg.Lattice, 'wcamg_lattice'), (wcamg.SetupParams, 'wcamg_setup_params'),
         (wcamg.SolveParams, 'wcamg_solve_params'), (wcamg.BicgParams, 'wcamg_bicg_params'),
         (wcamg.SolveInfo, 'wcamg_solve_info')]


def _c_layout(tmp_path):
    cc = shutil.which('gcc') or shutil.which('cc')
    if cc is None:
        pytest.skip('no host C compiler')
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "wcamg.h"', 'int main(void) {']
    for cls, cname in PAIRS:
        lines.append('printf("%s . %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ['return 0;', '}']
    src = tmp_path / 'layout.c'
    src.write_text('\n'.join(lines) + '\n')
    exe = tmp_path / 'layout'
    subprocess.run([cc, '-std=c99', '-I', INCLUDE, str(src), '-o', str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    return got


def test_ctypes_structs_match_the_header(tmp_path):
    got = _c_layout(tmp_path)
    import ctypes
    for cls, cname in PAIRS:
        assert ctypes.sizeof(cls) == got[(cname, '.')], cname
        for f in cls._fields_:
            assert getattr(cls, f[0]).offset == got[(cname, f[0])], (cname, f[0])


def _header_fields():
    """Field names of every typedef'd struct in the header, in order."""
    import re
    txt = re.sub(r'/\*.*?\*/', '', open(os.path.join(INCLUDE, 'wcamg.h')).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r'typedef struct\s*\{(.*?)\}\s*(\w+)\s*;', txt, flags=re.S):
        names = []
        for decl in body.split(';'):
            decl = re.sub(r'\[.*?\]', '', decl).strip()
            if decl:
                # "type a, b, c": the first part ends with a name, the rest are names
                parts = [q.strip() for q in decl.split(',')]
                names.append(parts[0].split()[-1].lstrip('*'))
                names.extend(q.lstrip('*') for q in parts[1:])
        out[name] = names
    return out


def test_binding_has_every_header_field_in_order():
    """Field names and order equal on both sides (a field missing from the
    binding could otherwise hide in a struct's tail padding)."""
    fields = _header_fields()
    for cls, cname in PAIRS:
        assert [f[0] for f in cls._fields_] == fields[cname], cname
