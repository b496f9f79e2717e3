"""Host-side logic that needs no GPU: the struct layouts the Python binding
marshals match the C header, and the served form's range allocator keeps
its invariants under random traffic (compiled natively with g++)."""
import ctypes
import os
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_2509_20776_amd", "csrc")


def _run_c(tmp_path, src, lang="c"):
    ext = "c" if lang == "c" else "cpp"
    f = tmp_path / f"t.{ext}"
    f.write_text(src)
    exe = tmp_path / "t"
    cc = ["gcc", "-std=c99"] if lang == "c" else ["g++", "-std=c++17", "-O1"]
    subprocess.run(cc + ["-I", INC, "-I", CSRC,
                         str(f), "-o", str(exe)], check=True, capture_output=True, text=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout


def test_struct_layouts_match_binding(tmp_path):
    from paper_2509_20776_amd import hipperm as hp
    structs = {"hp_csr_t": hp.hp_csr_t, "hp_dcsc_t": hp.hp_dcsc_t, "hp_plan_info_t": hp.hp_plan_info_t,
               "hp_request_t": hp.hp_request_t, "hp_batch_info_t": hp.hp_batch_info_t,
               "hp_server_config_t": hp.hp_server_config_t, "hp_completion_t": hp.hp_completion_t}
    lines = []
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"hipperm.h\"\nint main(void){\n" + \
          "\n".join(lines) + "\nreturn 0;}\n"
    got = {}
    for ln in _run_c(tmp_path, src).splitlines():
        a, b, c = ln.split()
        got[(a, b)] = int(c)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


def test_range_allocator_invariants(tmp_path):
    src = textwrap.dedent(r"""
        #include <cstdio>
        #include <cstdlib>
        #include <vector>
        #include <algorithm>
        #include "hp_alloc.hpp"
        using hp::RangeAlloc;
        struct B { size_t off, len; };
        static unsigned long long st = 12345;
        static unsigned rnd() { st = st * 6364136223846793005ull + 1442695040888963407ull; return (unsigned)(st >> 33); }
        int main() {
            const size_t cap = 1 << 24;
            RangeAlloc a(cap);
            std::vector<B> live;
            for (int it = 0; it < 200000; it++) {
                if (live.empty() || rnd() % 3) {
                    size_t n = rnd() % 3 ? rnd() % 4096 : rnd() % 400000;
                    size_t off = a.alloc(n);
                    if (off == RangeAlloc::NONE) { if (a.fits_now(n)) { puts("FAIL fits_now"); return 1; } continue; }
                    size_t len = RangeAlloc::round(n ? n : 1);
                    if (off % RangeAlloc::ALIGN || off + len > cap) { puts("FAIL range"); return 1; }
                    for (auto &b : live)
                        if (off < b.off + b.len && b.off < off + len) { puts("FAIL overlap"); return 1; }
                    live.push_back({off, len});
                } else {
                    size_t k = rnd() % live.size();
                    if (!a.release(live[k].off)) { puts("FAIL release"); return 1; }
                    if (a.release(live[k].off)) { puts("FAIL double release"); return 1; }
                    live.erase(live.begin() + k);
                }
                size_t sum = 0;
                for (auto &b : live) sum += b.len;
                if (sum != a.in_use() || a.blocks() != live.size()) { puts("FAIL accounting"); return 1; }
            }
            for (auto &b : live) a.release(b.off);
            if (a.in_use() != 0 || a.free_ranges() != 1 || !a.fits_now(cap) || a.fits_empty(cap + 1)) {
                puts("FAIL coalesce"); return 1;
            }
            printf("OK peak %zu\n", a.peak());
            return 0;
        }
    """)
    out = _run_c(tmp_path, src, lang="c++")
    assert out.startswith("OK"), out
