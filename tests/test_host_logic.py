"""Host-side logic that needs no GPU: the struct layouts the Python binding
marshals match the C header; the served form's range allocator keeps its
invariants under random traffic; the bounded host wait ends on completion,
on a failure and at its time limit, and stops spinning after its first
polls.  The C++ parts are compiled natively with g++, once plainly and once
with AddressSanitizer and UndefinedBehaviorSanitizer (host code only)."""
import ctypes
import os
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_2509_20776_amd", "csrc")


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _run_c(tmp_path, src, lang="c", flags=()):
    ext = "c" if lang == "c" else "cpp"
    f = tmp_path / f"t.{ext}"
    f.write_text(src)
    exe = tmp_path / "t"
    cc = ["gcc", "-std=c99"] if lang == "c" else ["g++", "-std=c++17", "-O1"]
    subprocess.run(cc + list(flags) + ["-I", INC, "-I", CSRC,
                                       str(f), "-o", str(exe)], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


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


@pytest.mark.parametrize("flags", [(), tuple(SANITIZE)], ids=["plain", "asan-ubsan"])
def test_range_allocator_invariants(tmp_path, flags):
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
    out = _run_c(tmp_path, src, lang="c++", flags=flags)
    assert out.startswith("OK"), out


@pytest.mark.parametrize("flags", [(), tuple(SANITIZE)], ids=["plain", "asan-ubsan"])
def test_bounded_wait(tmp_path, flags):
    """hp_poll.hpp driven by a fake query and a fake clock: it returns at
    completion or failure, times out at the limit, spins only for the first
    polls, then yields, then sleeps; the limit comes from HP_HOST_WAIT_MS."""
    src = textwrap.dedent(r"""
        #include <cstdio>
        #include <cstdlib>
        #include <vector>
        #include "hp_poll.hpp"
        using namespace hp;
        #define CHECK(c) do { if (!(c)) { printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
        int main() {
            WaitPolicy pol{50'000'000, 8, 16, 20'000};
            int64_t clock = 0;
            std::vector<int64_t> pauses;
            auto now = [&] { return clock; };
            auto pause = [&](int64_t ns) { pauses.push_back(ns); clock += ns > 0 ? ns : 100; };
            // ready at the 5th query: no pause inside the spin burst
            int q = 0;
            int64_t polls = 0;
            WaitResult r = wait_until([&] { return ++q >= 5 ? Poll::READY : Poll::PENDING; }, pol, now, pause, &polls);
            CHECK(r == WaitResult::DONE && polls == 5 && pauses.empty());
            // a failure ends the wait at once
            q = 0;
            r = wait_until([&] { return ++q >= 3 ? Poll::FAILED : Poll::PENDING; }, pol, now, pause, &polls);
            CHECK(r == WaitResult::FAILED && polls == 3);
            // never ready: spin burst, then yields, then sleeps, until the limit
            pauses.clear();
            clock = 0;
            r = wait_until([&] { clock += 1000; return Poll::PENDING; }, pol, now, pause, &polls);
            CHECK(r == WaitResult::TIMED_OUT);
            CHECK(clock >= pol.limit_ns && clock < pol.limit_ns + 2 * (pol.sleep_ns + 2000));
            CHECK(polls == (int64_t)pauses.size() + pol.spin_polls);
            for (size_t k = 0; k < pauses.size(); k++)
                CHECK(pauses[k] == (k < (size_t)pol.yield_polls ? 0 : pol.sleep_ns));
            // no limit: waits as long as it takes
            WaitPolicy forever{0, 2, 2, 1000};
            q = 0;
            r = wait_until([&] { return ++q >= 100000 ? Poll::READY : Poll::PENDING; }, forever, now, pause, &polls);
            CHECK(r == WaitResult::DONE && polls == 100000);
            // the real clock and pauses: a query that becomes ready after 3 ms
            const int64_t t0 = steady_ns();
            r = wait_until([&] { return steady_ns() - t0 > 3'000'000 ? Poll::READY : Poll::PENDING; },
                           default_wait_policy());
            CHECK(r == WaitResult::DONE);
            // and one that never does, with a 20 ms limit
            WaitPolicy short_pol = default_wait_policy();
            short_pol.limit_ns = 20'000'000;
            const int64_t t1 = steady_ns();
            r = wait_until([] { return Poll::PENDING; }, short_pol);
            CHECK(r == WaitResult::TIMED_OUT && steady_ns() - t1 >= 20'000'000);
            // the limit's source
            unsetenv("HP_HOST_WAIT_MS");
            CHECK(host_wait_limit_ns() == int64_t(600) * 1000000000);
            setenv("HP_HOST_WAIT_MS", "250", 1);
            CHECK(host_wait_limit_ns() == 250'000'000);
            setenv("HP_HOST_WAIT_MS", "zero", 1);
            CHECK(host_wait_limit_ns() == int64_t(600) * 1000000000);
            puts("OK");
            return 0;
        }
    """)
    out = _run_c(tmp_path, src, lang="c++", flags=flags)
    assert out.startswith("OK"), out


@pytest.mark.parametrize("flags", [(), tuple(SANITIZE)], ids=["plain", "asan-ubsan"])
def test_tuner_cache_file(tmp_path, flags):
    """hp_tunecache.hpp: the batched form's tuner choices round-trip through
    the cache file; later lines override earlier ones, malformed lines are
    skipped, keys with blanks are refused, the path follows HP_TUNE_CACHE and
    then XDG_CACHE_HOME, and a missing file reads as empty."""
    cache = tmp_path / "sub" / "tune.txt"
    src = textwrap.dedent(r"""
        #include <cstdio>
        #include <cstdlib>
        #include <string>
        #include "hp_tunecache.hpp"
        using namespace hp;
        #define CHECK(c) do { if (!(c)) { printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
        int main(int argc, char **argv) {
            const std::string path = argv[1];
            CHECK(tune_cache_load(path).empty());
            CHECK(tune_cache_store(path, "batch/cu256/plan/p0/v0/t2^10", 512));
            CHECK(tune_cache_store(path, "batch/cu256/exec/p0/v0/t2^12", 1024));
            CHECK(tune_cache_store(path, "batch/cu256/plan/p0/v0/t2^10", 256));
            CHECK(!tune_cache_store(path, "bad key", 3));
            CHECK(!tune_cache_store(path, "k", 0));
            FILE *f = fopen(path.c_str(), "a");
            fputs("garbage\n\n   \nnot_a_number x\n", f);
            fclose(f);
            auto m = tune_cache_load(path);
            CHECK(m.size() == 2);
            CHECK(m["batch/cu256/plan/p0/v0/t2^10"] == 256);
            CHECK(m["batch/cu256/exec/p0/v0/t2^12"] == 1024);
            setenv("HP_TUNE_CACHE", "/x/y.txt", 1);
            CHECK(tune_cache_path() == "/x/y.txt");
            setenv("HP_TUNE_CACHE", "", 1);
            CHECK(tune_cache_path().empty());
            CHECK(tune_cache_load(tune_cache_path()).empty() && !tune_cache_store(tune_cache_path(), "k", 1));
            unsetenv("HP_TUNE_CACHE");
            setenv("XDG_CACHE_HOME", "/c", 1);
            CHECK(tune_cache_path() == "/c/hipperm/batch_tune.txt");
            puts("OK");
            return 0;
        }
    """)
    f = tmp_path / "t.cpp"
    f.write_text(src)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-std=c++17", "-O1", *flags, "-I", CSRC, str(f), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    r = subprocess.run([str(exe), str(cache)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
