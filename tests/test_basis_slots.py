"""Host bookkeeping of the resident Krylov basis (csrc/basis_slots.h),
compiled from its header with g++ and driven on the CPU the way a run drives
it: an eager loop asks for slots 0..j before iteration j, the graph-replayed
loop for slots up to 2 L + 2 before launch L, and a call starts from the
chunks kept by earlier calls. Checked for every request: the launches cover
the new table entries exactly once and in order, each launch's entries lie in
the per_launch chunks it is given and in chunks that exist, the table covers
what was asked (never more than max_slots), and every slot's bytes lie inside
its chunk."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_11267_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "basis_slots.h"

static int fail(const char* what, int a, int b, int c) {
    std::printf("FAIL %s %d %d %d\n", what, a, b, c);
    return 1;
}

int main() {
    std::mt19937 rng(7);
    const int strides[] = {256, 356608, 25600000, 1 << 21};
    for (int trial = 0; trial < 4000; ++trial) {
        const size_t chunk_bytes = (trial % 3 == 0) ? (size_t(2) << 20) : (size_t(2048) << 20);
        const size_t stride = (size_t)strides[rng() % 4];
        if (stride > chunk_bytes) continue;
        const int per_chunk = (int)(chunk_bytes / stride);
        const int per_launch = 1 + (int)(rng() % 16);
        const int max_slots = 1 + (int)(rng() % 7000);
        const size_t pooled = rng() % 40;     // chunks kept from earlier calls
        size_t chunks = pooled;
        std::vector<int> covered(max_slots, 0);
        int cap = 0;
        auto request = [&](int slots) -> int {
            const int want = std::min(slots, max_slots);
            const size_t kend = want > cap ? ciq::basis_chunks_for(want, per_chunk) : 0;
            chunks = std::max(chunks, kend);                 // ensure() allocates these first
            int next = cap;
            int bad = 0;
            const int newcap = ciq::basis_table_ranges(cap, slots, per_chunk, max_slots, per_launch,
                                                       [&](int lo, int hi, int k0) {
                if (lo != next || hi <= lo) bad = 1;                       // in order, no gaps
                if (lo / per_chunk < k0 || (hi - 1) / per_chunk >= k0 + per_launch) bad = 2;
                if ((size_t)((hi - 1) / per_chunk) >= chunks) bad = 3;     // chunk exists
                for (int t = lo; t < hi; ++t) {
                    if (covered[t]++) bad = 4;                               // once
                    if ((size_t)(t % per_chunk + 1) * stride > chunk_bytes) bad = 5;
                }
                next = hi;
            });
            if (bad) return fail("range", bad, next, trial);
            if (newcap < cap || newcap < want || newcap > max_slots) return fail("cap", newcap, want, trial);
            if (newcap > cap && next != newcap) return fail("end", next, newcap, trial);
            cap = newcap;
            return 0;
        };
        // the call's set-up takes the pooled chunks, then the loop asks ahead
        if (request((int)std::min<size_t>(pooled * per_chunk, (size_t)max_slots))) return 1;
        const bool graph = trial & 1;
        for (int j = 1; j <= max_slots; j += 1 + (int)(rng() % 40)) {
            const int slots = graph ? 2 * ((j - 1) / 2) + 3 : j + 1;
            if (request(slots)) return 1;
        }
        if (request(max_slots + 5)) return 1;
        for (int t = 0; t < cap; ++t)
            if (covered[t] != 1) return fail("cover", t, cap, trial);
        if (cap != max_slots) return fail("final", cap, max_slots, trial);
    }
    std::printf("ok\n");
    return 0;
}
'''


def test_basis_table_ranges(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-I" + CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
