// Disk tier of the master mipmap ("Brick Upload from Disk to RAM", Fig. 5): the levels are cut
// into pages (a page holds the voxels of a cube of cells of one level, so several bricks'
// data travel together), the pages live in a file, and RAM holds an LRU set of them in fixed
// frames.  A page that was modified is written back before its frame is reused; a page that
// device work still uses cannot be removed -- the caller waits for that work to end (the
// paper's construction threads sleep until their brick arrives).
//
// Plain C++ and POSIX I/O, no device calls: the device side (which frames a batch of kernels
// uses, and when that batch has finished) comes in through `seq` numbers and two callbacks,
// so the policy is testable on the host alone.  The frames are either host memory the cache
// reads and writes directly, or memory it cannot address (device memory): then every page
// moves through a host staging buffer and three callbacks copy it in, copy it out and fill a
// frame with the background.
#pragma once

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

namespace octrc {

class PageCache {
public:
    struct Stats {
        uint64_t hits = 0;        // acquires of a resident page
        uint64_t loads = 0;       // pages read from the file into a frame
        uint64_t fills = 0;       // pages never written: frame filled with the background
        uint64_t writebacks = 0;  // modified pages written to the file before their frame was reused
        uint64_t evictions = 0;   // resident pages removed from RAM
        uint64_t waits = 0;       // evictions that had to wait for device work on the frame
        uint64_t bytes_read = 0, bytes_written = 0;
    };
    // wait(seq): block until the device work of batch seq (and every earlier one) has ended;
    // done(seq): whether it has ended, without blocking.
    using WaitFn = std::function<void(uint64_t)>;
    using DoneFn = std::function<bool(uint64_t)>;
    using FillFn = std::function<void(uint8_t *)>;
    // Frames the cache cannot address: load(f, src) copies a page from host memory into frame
    // f, store(f, dst) the frame's page into host memory, fill(f) fills frame f with the
    // background; each has finished when it returns (false: failed).  `staging` is a host
    // buffer of one page for the file I/O.
    struct FrameIO {
        std::function<bool(int, const uint8_t *)> load;
        std::function<bool(int, uint8_t *)> store;
        std::function<bool(int)> fill;
        uint8_t *staging = nullptr;
    };

    ~PageCache() { close(); }

    // Creates (truncates) the page file and takes `frames` (n_frames * page_bytes bytes of
    // host memory owned by the caller) as the RAM set.  Returns false with `err` set on failure.
    // `fill` fills a host page with the background.
    bool open(const std::string &path, int64_t n_pages, size_t page_bytes, uint8_t *frames,
              int n_frames, FillFn fill, std::string &err)
    {
        if (!frames) {
            err = "page cache: bad geometry";
            return false;
        }
        return open_impl(path, n_pages, page_bytes, frames, FrameIO{}, n_frames, std::move(fill), err);
    }

    // The same with n_frames frames that only `io` reaches.
    bool open(const std::string &path, int64_t n_pages, size_t page_bytes, FrameIO io,
              int n_frames, FillFn fill, std::string &err)
    {
        if (!io.load || !io.store || !io.fill || !io.staging) {
            err = "page cache: incomplete frame callbacks";
            return false;
        }
        return open_impl(path, n_pages, page_bytes, nullptr, std::move(io), n_frames,
                         std::move(fill), err);
    }

private:
    bool open_impl(const std::string &path, int64_t n_pages, size_t page_bytes, uint8_t *frames,
                   FrameIO io, int n_frames, FillFn fill, std::string &err)
    {
        close();
        if (n_pages < 1 || page_bytes == 0 || n_frames < 1) {
            err = "page cache: bad geometry";
            return false;
        }
        fd_ = ::open(path.c_str(), O_RDWR | O_CREAT | O_TRUNC, 0600);
        if (fd_ < 0) {
            err = "page cache: cannot create " + path + ": " + std::strerror(errno);
            return false;
        }
        path_ = path;
        page_bytes_ = page_bytes;
        frames_ = frames;
        fio_ = std::move(io);
        fill_ = std::move(fill);
        page_frame_.assign((size_t)n_pages, -1);
        on_disk_.assign((size_t)n_pages, 0);
        frame_page_.assign((size_t)n_frames, -1);
        dirty_.assign((size_t)n_frames, 0);
        stamp_.assign((size_t)n_frames, 0);
        last_seq_.assign((size_t)n_frames, 0);
        mark_.assign((size_t)n_frames, 0);
        clock_ = 0;
        stats = Stats();
        return true;
    }

public:
    // Closes and removes the page file (it only backs this process's octree).
    void close()
    {
        if (fd_ >= 0) {
            ::close(fd_);
            ::unlink(path_.c_str());
        }
        fd_ = -1;
    }

    int n_frames() const { return (int)frame_page_.size(); }
    int64_t n_pages() const { return (int64_t)page_frame_.size(); }
    size_t page_bytes() const { return page_bytes_; }
    int frame_of(int64_t page) const { return page_frame_[(size_t)page]; }
    bool device_frames() const { return frames_ == nullptr; }
    // host frames only
    uint8_t *frame_ptr(int f) const { return frames_ + (size_t)f * page_bytes_; }
    bool dirty(int f) const { return dirty_[(size_t)f] != 0; }
    bool on_disk(int64_t page) const { return on_disk_[(size_t)page] != 0; }

    // Makes every page of pages[0 .. n) resident for device batch `seq` (distinct pages, at most
    // n_frames of them).  Frames of this batch are never chosen as victims by it; among the
    // others the least recently used one whose device work has ended is taken, else the least
    // recently used one after waiting for its work.  write[i] (write may be NULL: none): the
    // batch modifies page i.  Returns 0, -1 when the pages do not fit in the frames, -2 on an
    // I/O error (err set).
    int acquire(const int64_t *pages, int n, const uint8_t *write, uint64_t seq,
                const WaitFn &wait, const DoneFn &done, std::string &err)
    {
        if (n > n_frames()) {
            err = "page cache: a batch needs " + std::to_string(n) + " pages, RAM holds " +
                  std::to_string(n_frames());
            return -1;
        }
        ++epoch_;
        for (int i = 0; i < n; i++) {   // the batch's resident pages first: they are not victims
            const int f = page_frame_[(size_t)pages[i]];
            if (f >= 0) mark_[(size_t)f] = epoch_;
        }
        for (int i = 0; i < n; i++) {
            const int64_t p = pages[i];
            int f = page_frame_[(size_t)p];
            if (f >= 0) {
                stats.hits++;
            } else {
                f = victim(done);
                if (frame_page_[(size_t)f] >= 0) {
                    if (!done(last_seq_[(size_t)f])) {
                        stats.waits++;
                        wait(last_seq_[(size_t)f]);
                    }
                    if (!evict(f, err)) return -2;
                }
                if (on_disk_[(size_t)p]) {
                    if (device_frames()) {
                        if (!io(false, p, fio_.staging, err)) return -2;
                        if (!fio_.load(f, fio_.staging)) return fail_frame("load", p, err);
                    } else if (!io(false, p, frame_ptr(f), err)) {
                        return -2;
                    }
                    stats.loads++;
                    stats.bytes_read += page_bytes_;
                } else {
                    if (device_frames()) {
                        if (!fio_.fill(f)) return fail_frame("fill", p, err);
                    } else {
                        fill_(frame_ptr(f));
                    }
                    stats.fills++;
                }
                frame_page_[(size_t)f] = p;
                page_frame_[(size_t)p] = f;
                dirty_[(size_t)f] = 0;
                mark_[(size_t)f] = epoch_;
            }
            stamp_[(size_t)f] = ++clock_;
            last_seq_[(size_t)f] = seq;
            if (write && write[i]) dirty_[(size_t)f] = 1;
        }
        return 0;
    }

    // Current contents of a page into dst (page_bytes): its frame (after its device work has
    // ended), else the file, else the background.
    bool read_page(int64_t p, uint8_t *dst, const WaitFn &wait, std::string &err)
    {
        const int f = page_frame_[(size_t)p];
        if (f >= 0) {
            wait(last_seq_[(size_t)f]);
            if (device_frames()) return fio_.store(f, dst) || fail_frame("read", p, err) == 0;
            std::memcpy(dst, frame_ptr(f), page_bytes_);
            return true;
        }
        if (on_disk_[(size_t)p]) return io(false, p, dst, err);
        fill_(dst);
        return true;
    }

    // Every page back to the background (the octree was cleared): frames are dropped without
    // write-back, after the device work on them has ended.
    void reset(const WaitFn &wait)
    {
        for (int f = 0; f < n_frames(); f++)
            if (frame_page_[(size_t)f] >= 0) {
                wait(last_seq_[(size_t)f]);
                page_frame_[(size_t)frame_page_[(size_t)f]] = -1;
                frame_page_[(size_t)f] = -1;
                dirty_[(size_t)f] = 0;
            }
        std::fill(on_disk_.begin(), on_disk_.end(), 0);
        if (fd_ >= 0 && ftruncate(fd_, 0) != 0) { /* a stale file tail is never read */ }
    }

    Stats stats;

private:
    int victim(const DoneFn &done)
    {
        int best = -1, best_idle = -1;
        for (int f = 0; f < n_frames(); f++) {
            if (mark_[(size_t)f] == epoch_) continue;     // used by this batch
            if (frame_page_[(size_t)f] < 0) return f;     // a free frame
            if (best < 0 || stamp_[(size_t)f] < stamp_[(size_t)best]) best = f;
            if ((best_idle < 0 || stamp_[(size_t)f] < stamp_[(size_t)best_idle]) &&
                done(last_seq_[(size_t)f]))
                best_idle = f;
        }
        return best_idle >= 0 ? best_idle : best;
    }

    bool evict(int f, std::string &err)
    {
        const int64_t p = frame_page_[(size_t)f];
        if (dirty_[(size_t)f]) {
            if (device_frames()) {
                if (!fio_.store(f, fio_.staging)) return fail_frame("write-back", p, err) == 0;
                if (!io(true, p, fio_.staging, err)) return false;
            } else if (!io(true, p, frame_ptr(f), err)) {
                return false;
            }
            on_disk_[(size_t)p] = 1;
            stats.writebacks++;
            stats.bytes_written += page_bytes_;
        }
        page_frame_[(size_t)p] = -1;
        frame_page_[(size_t)f] = -1;
        dirty_[(size_t)f] = 0;
        stats.evictions++;
        return true;
    }

    // -2 (an I/O error) with err set, for a failed frame copy or fill of page p
    static int fail_frame(const char *what, int64_t p, std::string &err)
    {
        err = std::string("page cache: frame ") + what + " of page " + std::to_string(p) + " failed";
        return -2;
    }

    bool io(bool wr, int64_t p, uint8_t *buf, std::string &err)
    {
        size_t done = 0;
        const off_t base = (off_t)p * (off_t)page_bytes_;
        while (done < page_bytes_) {
            const ssize_t r = wr ? ::pwrite(fd_, buf + done, page_bytes_ - done, base + (off_t)done)
                                 : ::pread(fd_, buf + done, page_bytes_ - done, base + (off_t)done);
            if (r < 0 && errno == EINTR) continue;
            if (r <= 0) {
                err = std::string("page cache: ") + (wr ? "write" : "read") + " of page " +
                      std::to_string(p) + " failed: " + (r < 0 ? std::strerror(errno) : "end of file");
                return false;
            }
            done += (size_t)r;
        }
        return true;
    }

    int fd_ = -1;
    std::string path_;
    size_t page_bytes_ = 0;
    uint8_t *frames_ = nullptr;   // host frames, or NULL: frames reached through fio_
    FrameIO fio_;
    FillFn fill_;
    std::vector<int32_t> page_frame_;   // frame holding each page, -1: not in RAM
    std::vector<uint8_t> on_disk_;      // the file holds the page's last written contents
    std::vector<int64_t> frame_page_;   // page in each frame, -1: free
    std::vector<uint8_t> dirty_;        // frame modified since it was loaded or filled
    std::vector<uint64_t> stamp_;       // last use (LRU clock)
    std::vector<uint64_t> last_seq_;    // last device batch that used the frame
    std::vector<uint64_t> mark_;        // epoch of the batch being acquired
    uint64_t clock_ = 0, epoch_ = 0;
};

}  // namespace octrc
