// Field files: a device field streamed to and from NumPy .npy files (format
// version 1.0 written; 1.0, 2.0 and 3.0 read), in place of the MATLAB files
// that the paper's end-to-end run writes for its initial and final
// concentrations (Sec. 5.3).  The bytes move through two pinned host buffers
// held by the grid: while one chunk is copied between the device and one
// buffer on the grid's stream, the other buffer is written to (or read from)
// the file, so the device copy and the file I/O overlap.
#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace {

constexpr size_t kIoChunk = (size_t)32 << 20;   // bytes per pinned buffer

int io_fail(int code, const std::string& msg)
{
    bfvm::set_error(msg);
    return code;
}

int hip_io_fail(hipError_t e, const char* what)
{
    return io_fail(e == hipErrorOutOfMemory ? BFVM_ENOMEM : BFVM_EDEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

#define IO_HIP(expr, what)                              \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_io_fail(_e, what); \
    } while (0)

const char* npy_descr(int dtype) { return dtype == BFVM_F64 ? "<f8" : "<f4"; }

// The pinned buffers and their events, allocated on first use.
int ensure_io_buffers(bfvm_grid g)
{
    if (g->io_buf[0]) return BFVM_OK;
    for (int b = 0; b < 2; ++b) {
        IO_HIP(hipHostMalloc(&g->io_buf[b], kIoChunk, hipHostMallocDefault), "hipHostMalloc");
        IO_HIP(hipEventCreateWithFlags(&g->io_ev[b], hipEventDisableTiming), "hipEventCreate");
    }
    return BFVM_OK;
}

struct File {
    FILE* f = nullptr;
    ~File()
    {
        if (f) std::fclose(f);
    }
};

std::string header_dict(bfvm_grid g)
{
    std::string d = std::string("{'descr': '") + npy_descr(g->dtype) + "', 'fortran_order': False, 'shape': (" +
                    std::to_string(g->nz) + ", " + std::to_string(g->ny) + ", " + std::to_string(g->nx) + ", " +
                    std::to_string(g->S) + "), }";
    // magic (6) + version (2) + length (2) + dict + newline: a multiple of 64
    const size_t used = 10 + d.size() + 1;
    d.append((64 - used % 64) % 64, ' ');
    d.push_back('\n');
    return d;
}

// Value text after "'key':" in the header dict (empty if absent).
std::string dict_value(const std::string& h, const char* key)
{
    const std::string k = std::string("'") + key + "'";
    size_t p = h.find(k);
    if (p == std::string::npos) return "";
    p = h.find(':', p + k.size());
    if (p == std::string::npos) return "";
    ++p;
    while (p < h.size() && h[p] == ' ') ++p;
    if (p >= h.size()) return "";
    if (h[p] == '\'' || h[p] == '"') {
        const size_t q = h.find(h[p], p + 1);
        return q == std::string::npos ? "" : h.substr(p + 1, q - p - 1);
    }
    if (h[p] == '(') {
        const size_t q = h.find(')', p);
        return q == std::string::npos ? "" : h.substr(p, q - p + 1);
    }
    size_t q = p;
    while (q < h.size() && h[q] != ',' && h[q] != '}') ++q;
    return h.substr(p, q - p);
}

// "(a, b, c)" -> integers; false if malformed
bool parse_shape(const std::string& s, std::vector<int64_t>& out)
{
    out.clear();
    if (s.size() < 2 || s.front() != '(' || s.back() != ')') return false;
    size_t p = 1;
    while (p < s.size() - 1) {
        while (p < s.size() - 1 && (s[p] == ' ' || s[p] == ',')) ++p;
        if (p >= s.size() - 1) break;
        if (s[p] < '0' || s[p] > '9') return false;
        int64_t v = 0;
        while (p < s.size() - 1 && s[p] >= '0' && s[p] <= '9') {
            if (v > (int64_t)1 << 40) return false;
            v = v * 10 + (s[p] - '0');
            ++p;
        }
        out.push_back(v);
    }
    return true;
}

}  // namespace

int bfvm_save_npy(bfvm_grid g, const void* field, const char* path)
{
    if (!g) return io_fail(BFVM_EINVAL, "grid is NULL");
    if (!field || !path) return io_fail(BFVM_EINVAL, "NULL pointer");
    File f;
    f.f = std::fopen(path, "wb");
    if (!f.f) return io_fail(BFVM_EIO, std::string("cannot open ") + path + " for writing: " + std::strerror(errno));
    const std::string dict = header_dict(g);
    unsigned char pre[10] = {0x93, 'N', 'U', 'M', 'P', 'Y', 1, 0, (unsigned char)(dict.size() & 0xff),
                             (unsigned char)(dict.size() >> 8)};
    if (std::fwrite(pre, 1, 10, f.f) != 10 || std::fwrite(dict.data(), 1, dict.size(), f.f) != dict.size())
        return io_fail(BFVM_EIO, std::string("write failed: ") + path);
    if (int st = ensure_io_buffers(g)) return st;
    const size_t total = (size_t)g->nelem() * bfvm::dtype_size(g->dtype);
    const char* src = static_cast<const char*>(field);
    const size_t nchunk = (total + kIoChunk - 1) / kIoChunk;
    // chunk i goes to buffer i % 2; the file write of chunk i - 1 overlaps
    // the device copy of chunk i
    for (size_t i = 0; i <= nchunk; ++i) {
        if (i < nchunk) {
            const size_t off = i * kIoChunk, len = std::min(kIoChunk, total - off);
            IO_HIP(hipMemcpyAsync(g->io_buf[i % 2], src + off, len, hipMemcpyDeviceToHost, g->stream),
                   "hipMemcpyAsync");
            IO_HIP(hipEventRecord(g->io_ev[i % 2], g->stream), "hipEventRecord");
        }
        if (i > 0) {
            const size_t j = i - 1, off = j * kIoChunk, len = std::min(kIoChunk, total - off);
            IO_HIP(hipEventSynchronize(g->io_ev[j % 2]), "hipEventSynchronize");
            if (std::fwrite(g->io_buf[j % 2], 1, len, f.f) != len) {
                // the copy of chunk i may still be filling the other pinned
                // buffer, which the next save or load on this grid reuses
                (void)hipStreamSynchronize(g->stream);
                return io_fail(BFVM_EIO, std::string("write failed: ") + path);
            }
        }
    }
    const int closed = std::fclose(f.f);
    f.f = nullptr;
    if (closed != 0) return io_fail(BFVM_EIO, std::string("close failed: ") + path);
    return BFVM_OK;
}

int bfvm_load_npy(bfvm_grid g, void* field, const char* path)
{
    if (!g) return io_fail(BFVM_EINVAL, "grid is NULL");
    if (!field || !path) return io_fail(BFVM_EINVAL, "NULL pointer");
    File f;
    f.f = std::fopen(path, "rb");
    if (!f.f) return io_fail(BFVM_EIO, std::string("cannot open ") + path + ": " + std::strerror(errno));
    unsigned char pre[8];
    if (std::fread(pre, 1, 8, f.f) != 8 || std::memcmp(pre, "\x93NUMPY", 6) != 0)
        return io_fail(BFVM_EINVAL, std::string(path) + " is not a .npy file");
    const int major = pre[6];
    if (major < 1 || major > 3) return io_fail(BFVM_EINVAL, "unsupported .npy version " + std::to_string(major));
    size_t hlen = 0;
    unsigned char lb[4] = {0, 0, 0, 0};
    const size_t nlb = major == 1 ? 2 : 4;
    if (std::fread(lb, 1, nlb, f.f) != nlb) return io_fail(BFVM_EINVAL, "truncated .npy header");
    hlen = (size_t)lb[0] | ((size_t)lb[1] << 8) | ((size_t)lb[2] << 16) | ((size_t)lb[3] << 24);
    if (hlen == 0 || hlen > (1u << 20)) return io_fail(BFVM_EINVAL, "bad .npy header length");
    std::string h(hlen, '\0');
    if (std::fread(&h[0], 1, hlen, f.f) != hlen) return io_fail(BFVM_EINVAL, "truncated .npy header");
    const std::string descr = dict_value(h, "descr");
    if (descr != npy_descr(g->dtype))
        return io_fail(BFVM_EINVAL, "element type '" + descr + "' does not match the grid's '" +
                                        npy_descr(g->dtype) + "'");
    if (dict_value(h, "fortran_order") != "False") return io_fail(BFVM_EINVAL, "Fortran-ordered arrays are not read");
    std::vector<int64_t> shape;
    if (!parse_shape(dict_value(h, "shape"), shape)) return io_fail(BFVM_EINVAL, "malformed shape in .npy header");
    const bool full = shape.size() == 4 && shape[0] == g->nz && shape[1] == g->ny && shape[2] == g->nx &&
                      shape[3] == g->S;
    const bool flat = g->S == 1 && shape.size() == 3 && shape[0] == g->nz && shape[1] == g->ny && shape[2] == g->nx;
    if (!full && !flat) return io_fail(BFVM_EINVAL, "array shape does not match the grid (nz, ny, nx, nsub)");
    const size_t total = (size_t)g->nelem() * bfvm::dtype_size(g->dtype);
    const long data0 = std::ftell(f.f);
    if (data0 < 0 || std::fseek(f.f, 0, SEEK_END) != 0) return io_fail(BFVM_EIO, "seek failed");
    const long end = std::ftell(f.f);
    if (end < 0 || (size_t)(end - data0) != total) return io_fail(BFVM_EINVAL, "file size does not match the shape");
    if (std::fseek(f.f, data0, SEEK_SET) != 0) return io_fail(BFVM_EIO, "seek failed");
    if (int st = ensure_io_buffers(g)) return st;
    char* dst = static_cast<char*>(field);
    const size_t nchunk = (total + kIoChunk - 1) / kIoChunk;
    // chunk i is read into buffer i % 2 once the device copy of chunk i - 2
    // (the buffer's previous contents) has finished
    for (size_t i = 0; i < nchunk; ++i) {
        const size_t off = i * kIoChunk, len = std::min(kIoChunk, total - off);
        if (i >= 2) IO_HIP(hipEventSynchronize(g->io_ev[i % 2]), "hipEventSynchronize");
        if (std::fread(g->io_buf[i % 2], 1, len, f.f) != len) {
            // copies still in flight read the pinned buffers that the next
            // call refills from the host
            (void)hipStreamSynchronize(g->stream);
            return io_fail(BFVM_EIO, std::string("read failed: ") + path);
        }
        IO_HIP(hipMemcpyAsync(dst + off, g->io_buf[i % 2], len, hipMemcpyHostToDevice, g->stream),
               "hipMemcpyAsync");
        IO_HIP(hipEventRecord(g->io_ev[i % 2], g->stream), "hipEventRecord");
    }
    IO_HIP(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    return BFVM_OK;
}
