// Storage side of the chunk pipeline (paper, Section 2.3: reading data chunks
// from the storage drive and writing reconstructed chunks back run in their
// own threads, in parallel, overlapped with the CPU-GPU transfers and the GPU
// computation).  Host code only; implements the tp_io_* calls of include/tp.h.
//
// A chunk of detector rows [z0, z1) of a projection-major file
// [n_outer][n_rows][n_det] (n_outer = angles, or dark/flat frames) is n_outer
// strided pieces of (z1 - z0) * n_det elements; the pieces are split over
// threads that each issue pread() calls.  Slices of the reconstruction are
// contiguous in the output file and are written with pwrite() the same way.
// When the file offsets, the lengths and the host buffer are 4096-byte aligned
// the file is opened with O_DIRECT, so the transfer does not pass through the
// page cache (the measured rate is the drive's, not RAM's); a buffer the
// kernel cannot pin for the transfer goes through per-thread aligned bounce
// buffers (still direct); a filesystem that refuses direct transfers gets
// buffered I/O.
#ifndef _GNU_SOURCE
#define _GNU_SOURCE
#endif
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tp.h"

namespace {

constexpr int64_t kAlign = 4096;
constexpr int kMaxThreads = 64;

thread_local std::string g_io_err;

tp_status io_fail(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_io_err = buf;
    return TP_EINVAL;
}

bool aligned(int64_t v) { return (v % kAlign) == 0; }

// Read or write `len` bytes at `off`, looping over short transfers.
bool full_io(int fd, char* buf, int64_t len, int64_t off, bool write, int* err) {
    while (len > 0) {
        const ssize_t r = write ? pwrite(fd, buf, static_cast<size_t>(len), off)
                                : pread(fd, buf, static_cast<size_t>(len), off);
        if (r < 0) {
            if (errno == EINTR) continue;
            *err = errno;
            return false;
        }
        if (r == 0) {  // end of file while reading
            *err = 0;
            return false;
        }
        buf += r;
        off += r;
        len -= r;
    }
    return true;
}

struct Piece {
    int64_t file_off, buf_off, len;
};

// How a call moves its pieces.
enum class Mode {
    kBuffered,      // through the page cache
    kDirect,        // O_DIRECT into / out of the caller's buffer
    kDirectBounce,  // O_DIRECT through a per-thread aligned buffer plus a memcpy
};
constexpr int64_t kBounceBytes = int64_t{16} << 20;

// Runs the pieces on n_threads threads; on failure *err_no holds the errno
// (0 for a file that is too short).
tp_status run_pieces_once(const char* path, bool write, char* buf, const std::vector<Piece>& pieces, int n_threads,
                          Mode mode, int* err_no, bool* open_failed) {
    *err_no = 0;
    *open_failed = false;
    const int flags = (write ? O_WRONLY : O_RDONLY) | (mode == Mode::kBuffered ? 0 : O_DIRECT);
    const int fd = open(path, flags);
    if (fd < 0) {
        *err_no = errno;
        *open_failed = true;
        return TP_EINVAL;
    }
    std::atomic<size_t> next{0};
    std::atomic<int> failed{0}, fail_errno{0};
    auto worker = [&]() {
        char* bounce = nullptr;
        if (mode == Mode::kDirectBounce) {
            void* p = nullptr;
            if (posix_memalign(&p, static_cast<size_t>(kAlign), static_cast<size_t>(kBounceBytes)) != 0) {
                fail_errno.store(ENOMEM);
                failed.store(1);
                return;
            }
            bounce = static_cast<char*>(p);
        }
        for (;;) {
            const size_t i = next.fetch_add(1);
            if (i >= pieces.size() || failed.load()) break;
            const Piece& pc = pieces[i];
            int e = 0;
            bool ok = true;
            if (bounce == nullptr) {
                ok = full_io(fd, buf + pc.buf_off, pc.len, pc.file_off, write, &e);
            } else {
                for (int64_t done = 0; ok && done < pc.len; done += kBounceBytes) {
                    const int64_t n = std::min(kBounceBytes, pc.len - done);
                    if (write) {
                        std::memcpy(bounce, buf + pc.buf_off + done, static_cast<size_t>(n));
                        ok = full_io(fd, bounce, n, pc.file_off + done, true, &e);
                    } else {
                        ok = full_io(fd, bounce, n, pc.file_off + done, false, &e);
                        if (ok) std::memcpy(buf + pc.buf_off + done, bounce, static_cast<size_t>(n));
                    }
                }
            }
            if (!ok) {
                fail_errno.store(e);
                failed.store(1);
                break;
            }
        }
        free(bounce);
    };
    const int nt = std::max(1, std::min({n_threads, kMaxThreads, static_cast<int>(pieces.size())}));
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) th.emplace_back(worker);
    for (auto& t : th) t.join();
    close(fd);
    if (failed.load()) {
        *err_no = fail_errno.load();
        return TP_EINVAL;
    }
    return TP_OK;
}

// Aligned transfers go direct; a buffer the kernel cannot pin for a direct
// transfer (EFAULT: e.g. the GPU runtime's pinned host memory) goes through
// bounce buffers; a filesystem that refuses direct transfers (EINVAL at open
// or transfer) gets buffered I/O.
tp_status run_pieces(const char* path, bool write, char* buf, const std::vector<Piece>& pieces, int n_threads,
                     bool try_direct) {
    int e = 0;
    bool open_failed = false;
    Mode mode = try_direct ? Mode::kDirect : Mode::kBuffered;
    tp_status st = run_pieces_once(path, write, buf, pieces, n_threads, mode, &e, &open_failed);
    if (st != TP_OK && mode == Mode::kDirect && e == EFAULT) {
        mode = Mode::kDirectBounce;
        st = run_pieces_once(path, write, buf, pieces, n_threads, mode, &e, &open_failed);
    }
    if (st != TP_OK && mode != Mode::kBuffered && e == EINVAL) {
        mode = Mode::kBuffered;
        st = run_pieces_once(path, write, buf, pieces, n_threads, mode, &e, &open_failed);
    }
    if (st != TP_OK && open_failed) return io_fail("cannot open %s: %s", path, strerror(e));
    if (st != TP_OK) {
        const char* how = mode == Mode::kBuffered ? "" : (mode == Mode::kDirect ? " (O_DIRECT)" : " (O_DIRECT, bounce)");
        return io_fail("%s %s failed%s: %s", write ? "writing" : "reading", path, how,
                       e ? strerror(e) : "file too short");
    }
    return TP_OK;
}

}  // namespace

extern "C" {

const char* tp_io_last_error(void) { return g_io_err.c_str(); }

tp_status tp_io_read_rows(const char* path, int64_t header_bytes, int32_t n_outer, int32_t n_rows, int32_t n_det,
                          int32_t z0, int32_t z1, int32_t elem_bytes, void* dst, int32_t n_threads) {
    if (!path || !dst) return io_fail("null path or buffer");
    if (n_outer <= 0 || n_rows <= 0 || n_det <= 0 || elem_bytes <= 0 || header_bytes < 0)
        return io_fail("sizes must be positive (n_outer=%d n_rows=%d n_det=%d elem_bytes=%d)", n_outer, n_rows,
                       n_det, elem_bytes);
    if (z0 < 0 || z1 <= z0 || z1 > n_rows) return io_fail("row range [%d, %d) outside [0, %d)", z0, z1, n_rows);
    const int64_t row = static_cast<int64_t>(n_det) * elem_bytes;
    const int64_t piece = static_cast<int64_t>(z1 - z0) * row;
    std::vector<Piece> pieces(static_cast<size_t>(n_outer));
    bool direct = aligned(reinterpret_cast<intptr_t>(dst)) && aligned(piece);
    for (int32_t o = 0; o < n_outer; ++o) {
        const int64_t off = header_bytes + (static_cast<int64_t>(o) * n_rows + z0) * row;
        pieces[static_cast<size_t>(o)] = Piece{off, static_cast<int64_t>(o) * piece, piece};
        direct = direct && aligned(off);
    }
    return run_pieces(path, false, static_cast<char*>(dst), pieces, n_threads, direct);
}

tp_status tp_io_write_slices(const char* path, int64_t header_bytes, int64_t first_slice, int32_t n_slices,
                             int64_t slice_bytes, const void* src, int32_t n_threads) {
    if (!path || !src) return io_fail("null path or buffer");
    if (n_slices <= 0 || slice_bytes <= 0 || first_slice < 0 || header_bytes < 0)
        return io_fail("bad slice range (first=%lld n=%d bytes=%lld)", static_cast<long long>(first_slice), n_slices,
                       static_cast<long long>(slice_bytes));
    std::vector<Piece> pieces(static_cast<size_t>(n_slices));
    bool direct = aligned(reinterpret_cast<intptr_t>(src)) && aligned(slice_bytes) && aligned(header_bytes);
    for (int32_t s = 0; s < n_slices; ++s)
        pieces[static_cast<size_t>(s)] =
            Piece{header_bytes + (first_slice + s) * slice_bytes, static_cast<int64_t>(s) * slice_bytes, slice_bytes};
    const tp_status st = run_pieces(path, true, static_cast<char*>(const_cast<void*>(src)), pieces, n_threads, direct);
    if (st != TP_OK) return st;
    // Start writing the range out now (without waiting): buffered writes would
    // otherwise sit in the page cache until a final flush, and the drive would
    // not work while later chunks are read and reconstructed.
    const int fd = open(path, O_WRONLY);
    if (fd >= 0) {
        (void)sync_file_range(fd, header_bytes + first_slice * slice_bytes,
                              static_cast<int64_t>(n_slices) * slice_bytes, SYNC_FILE_RANGE_WRITE);
        close(fd);
    }
    return TP_OK;
}

tp_status tp_io_create(const char* path, int64_t bytes) {
    if (!path || bytes < 0) return io_fail("null path or negative size");
    const int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (fd < 0) return io_fail("cannot create %s: %s", path, strerror(errno));
    const int r = ftruncate(fd, bytes);
    const int e = errno;
    close(fd);
    if (r != 0) return io_fail("cannot size %s to %lld bytes: %s", path, static_cast<long long>(bytes), strerror(e));
    return TP_OK;
}

}  // extern "C"
