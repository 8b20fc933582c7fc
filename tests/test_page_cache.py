"""Host-only checks of the disk tier's page cache (LRU frames over a page file, write-back of
modified pages, pages pinned by device work in flight): a small C++ driver includes the
library's page_cache.h, plays scripted batches against it with a simulated device, and prints
one line per check.  It runs twice: with host frames the cache addresses itself, and with
frames only reachable through copy and fill callbacks (as device frames are), whose copies go
through a host staging buffer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1407_2074_amd", "csrc")

DRIVER = r"""
#include "page_cache.h"
#include <cstdio>
#include <set>
using namespace octrc;

static std::set<uint64_t> running;          // device batches not yet finished
static std::vector<uint64_t> waited;        // batches the cache waited for
static void check(const char *name, bool ok) { std::printf("%s %d\n", name, ok ? 1 : 0); }

int main(int argc, char **argv)
{
    const size_t PB = 64;                   // bytes per page
    const bool devmode = argc > 2;          // frames reached only through the callbacks
    std::vector<uint8_t> frames(4 * PB), staging(PB);
    PageCache pc;
    std::string err;
    auto fill = [](uint8_t *f) { std::fill_n(f, 64, (uint8_t)7); };
    static int copies_in = 0, copies_out = 0;
    bool opened;
    if (devmode) {
        PageCache::FrameIO io;
        io.load = [&](int f, const uint8_t *src) {
            copies_in++;
            std::memcpy(frames.data() + f * PB, src, PB);
            return src == staging.data();
        };
        io.store = [&](int f, uint8_t *dst) {
            copies_out++;
            std::memcpy(dst, frames.data() + f * PB, PB);
            return true;
        };
        io.fill = [&](int f) { std::fill_n(frames.data() + f * PB, PB, (uint8_t)7); return true; };
        io.staging = staging.data();
        opened = pc.open(argv[1], 16, PB, io, 4, fill, err);
    } else {
        opened = pc.open(argv[1], 16, PB, frames.data(), 4, fill, err);
    }
    if (!opened) { std::printf("open %s\n", err.c_str()); return 1; }
    check("mode", pc.device_frames() == devmode);
    auto fp = [&](int f) { return frames.data() + (size_t)f * PB; };   // the frames' memory
    PageCache::WaitFn wait = [](uint64_t q) {
        waited.push_back(q);
        for (auto it = running.begin(); it != running.end();) it = *it <= q ? running.erase(it) : ++it;
    };
    PageCache::DoneFn done = [](uint64_t q) { return running.empty() || *running.begin() > q; };
    auto put = [&](int64_t p, uint8_t v) { std::fill_n(fp(pc.frame_of(p)), PB, v); };

    // batch 1 writes pages 0..3 (fills: never written before)
    const int64_t a[4] = {0, 1, 2, 3};
    const uint8_t w1[4] = {1, 1, 1, 1};
    check("fit", pc.acquire(a, 4, w1, 1, wait, done, err) == 0);
    for (int64_t p = 0; p < 4; p++) put(p, (uint8_t)(100 + p));
    check("fills4", pc.stats.fills == 4 && pc.stats.loads == 0);
    // batch 2 reads page 4 while batch 1 has ended: LRU page 0 is written back and evicted
    const int64_t b[1] = {4};
    check("acquire_b", pc.acquire(b, 1, nullptr, 2, wait, done, err) == 0);
    check("lru_victim_is_page0", pc.frame_of(0) < 0 && pc.frame_of(1) >= 0);
    check("writeback1", pc.stats.writebacks == 1 && pc.stats.evictions == 1 && pc.on_disk(0));
    check("no_wait_when_idle", pc.stats.waits == 0 && waited.empty());
    // page 0 comes back from the file with what batch 1 wrote
    const int64_t c[1] = {0};
    check("acquire_c", pc.acquire(c, 1, nullptr, 3, wait, done, err) == 0);
    check("reload_contents", fp(pc.frame_of(0))[0] == 100 && pc.stats.loads == 1);
    // page 1 (LRU) went out, written back; page 4 was only read: evicting it writes nothing
    check("writeback2", pc.stats.writebacks == 2);
    // batch 5 is in flight on pages 2, 3 (touched last): a victim is taken among idle frames
    running.insert(5);
    const int64_t d[2] = {2, 3};
    check("acquire_d", pc.acquire(d, 2, nullptr, 5, wait, done, err) == 0);
    const int64_t e[1] = {9};
    check("acquire_e", pc.acquire(e, 1, nullptr, 6, wait, done, err) == 0);
    check("busy_pages_kept", pc.frame_of(2) >= 0 && pc.frame_of(3) >= 0 && waited.empty());
    // every other frame busy too: the cache waits for the oldest batch on the LRU frame
    running.insert(6);
    running.insert(7);
    const int64_t f7[1] = {0};
    check("acquire_f", pc.acquire(f7, 1, nullptr, 7, wait, done, err) == 0);
    const int64_t g8[1] = {10};
    check("acquire_g", pc.acquire(g8, 1, nullptr, 8, wait, done, err) == 0);
    check("waited_for_busy", pc.stats.waits == 1 && waited.size() == 1 && waited[0] == 5);
    // a batch never evicts its own pages; more pages than frames is refused
    const int64_t h4[4] = {11, 12, 13, 14};
    check("own_pages", pc.acquire(h4, 4, nullptr, 9, wait, done, err) == 0 &&
                           pc.frame_of(11) >= 0 && pc.frame_of(12) >= 0 && pc.frame_of(13) >= 0 &&
                           pc.frame_of(14) >= 0);
    const int64_t i5[5] = {0, 1, 2, 3, 4};
    check("too_many", pc.acquire(i5, 5, nullptr, 10, wait, done, err) == -1);
    // read_page: from the file, from a frame, or the background
    std::vector<uint8_t> buf(PB);
    check("read_disk", pc.read_page(1, buf.data(), wait, err) && buf[0] == 101);
    check("read_never", pc.read_page(15, buf.data(), wait, err) && buf[0] == 7);
    put(11, 42);
    check("read_frame", pc.read_page(11, buf.data(), wait, err) && buf[0] == 42);
    // reset: everything back to the background, nothing written back
    const uint64_t wb = pc.stats.writebacks;
    pc.reset(wait);
    check("reset_background", pc.read_page(0, buf.data(), wait, err) && buf[0] == 7 &&
                                  pc.frame_of(11) < 0 && pc.stats.writebacks == wb);
    // the callbacks carried every page in and out (device frames): one copy in per load, one
    // copy out per write-back and per frame read
    check("frame_copies", !devmode || (copies_in == (int)pc.stats.loads &&
                                       copies_out == (int)pc.stats.writebacks + 1));
    pc.close();
    check("file_removed", access(argv[1], F_OK) != 0);
    return 0;
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    d = tmp_path_factory.mktemp("pagecache")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, "-o", str(exe), str(src)])
    res = {}
    for mode, extra in (("host", []), ("device", ["device"])):
        out = subprocess.run([str(exe), str(d / f"pages_{mode}.bin")] + extra, capture_output=True,
                             text=True, check=True).stdout
        res[mode] = dict(line.split() for line in out.splitlines())
    return res


@pytest.mark.parametrize("mode", ["host", "device"])
@pytest.mark.parametrize("name", [
    "mode", "fit", "fills4", "acquire_b", "lru_victim_is_page0", "writeback1",
    "no_wait_when_idle", "acquire_c", "reload_contents", "writeback2", "acquire_d", "acquire_e",
    "busy_pages_kept", "acquire_f", "acquire_g", "waited_for_busy", "own_pages", "too_many",
    "read_disk", "read_never", "read_frame", "reset_background", "frame_copies",
    "file_removed"])
def test_page_cache(results, mode, name):
    assert results[mode].get(name) == "1", (mode, name, results[mode])
