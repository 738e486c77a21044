// Model files: the fitted operator (lambda, b, Sigma, mode kinds, modes Phi) stored once
// after the offline fit and loaded by the run-time evaluation (Sec. 4.4: the reduced model
// is precomputed, then stepped or evaluated in one product per frame).
//
// Layout (little-endian, 64-byte header, then the payload):
//   0  char[8]  magic "DMDMODEL"
//   8  u32      format version (1)
//  12  u32      header bytes (64)
//  16  i64      N (rows of Phi)
//  24  i32      r (modes)
//  28  i32      dtype of Phi (0 FP32, 1 FP64)
//  32  f64      dt
//  40  u64      payload bytes
//  48  u64      FNV-1a 64 hash of the payload
//  56  u32      ABI version of the writer
//  60  u32      reserved (0)
// payload: lam (2r f64, interleaved re/im), b (2r f64), sigma (r f64), kind (r i32),
//          Phi (N x r, row-major, the model's dtype; the padding columns are not stored).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "dmdmi.h"

namespace {

constexpr char MAGIC[8] = {'D', 'M', 'D', 'M', 'O', 'D', 'E', 'L'};
constexpr uint32_t FORMAT_VERSION = 1;
constexpr uint32_t HEADER_BYTES = 64;
constexpr int64_t ROW_CHUNK = 65536;   // rows of Phi staged through host memory at a time

struct Header {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    int64_t n;
    int32_t r;
    int32_t dtype;
    double dt;
    uint64_t payload_bytes;
    uint64_t hash;
    uint32_t abi;
    uint32_t reserved;
};
static_assert(sizeof(Header) == HEADER_BYTES, "model file header is 64 bytes");

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    }
};

uint64_t payload_bytes(int64_t n, int32_t r, int32_t dtype)
{
    const uint64_t esz = dtype == DMD_F64 ? 8 : 4;
    return (uint64_t)r * (2 * 8 + 2 * 8 + 8 + 4) + (uint64_t)n * (uint64_t)r * esz;
}

struct File {
    FILE* f = nullptr;
    ~File() { if (f) fclose(f); }
};

// Reads and checks the header and (with check_hash) the payload hash; leaves the file
// positioned at the payload.
int32_t read_header(FILE* f, Header* h, bool check_hash)
{
    if (fread(h, 1, sizeof(Header), f) != sizeof(Header)) return DMD_ERR_IO;
    if (memcmp(h->magic, MAGIC, 8) != 0) return DMD_ERR_IO;
    if (h->version != FORMAT_VERSION || h->header_bytes != HEADER_BYTES) return DMD_ERR_IO;
    if (h->n < 1 || h->r < 1 || (h->dtype != DMD_F32 && h->dtype != DMD_F64)) return DMD_ERR_IO;
    if (!(h->dt > 0.0) || h->dt != h->dt) return DMD_ERR_IO;
    if (h->payload_bytes != payload_bytes(h->n, h->r, h->dtype)) return DMD_ERR_IO;
    if (check_hash) {
        Fnv fnv;
        std::vector<unsigned char> buf(1 << 20);
        uint64_t left = h->payload_bytes;
        while (left > 0) {
            const size_t want = (size_t)std::min<uint64_t>(left, buf.size());
            if (fread(buf.data(), 1, want, f) != want) return DMD_ERR_IO;
            fnv.add(buf.data(), want);
            left -= want;
        }
        if (fgetc(f) != EOF) return DMD_ERR_IO;   // trailing bytes
        if (fnv.h != h->hash) return DMD_ERR_IO;
        if (fseek(f, (long)HEADER_BYTES, SEEK_SET) != 0) return DMD_ERR_IO;
    }
    return DMD_OK;
}

}  // namespace

#define HIPCHK_IO(x)                                \
    do {                                            \
        if ((x) != hipSuccess) return DMD_ERR_HIP;  \
    } while (0)

extern "C" {

int32_t dmd_model_file_info(const char* path, int64_t* n, int32_t* r, int32_t* dtype, double* dt)
{
    if (!path || !n || !r || !dtype || !dt) return DMD_ERR_ARG;
    File F;
    F.f = fopen(path, "rb");
    if (!F.f) return DMD_ERR_IO;
    Header h;
    if (int32_t e = read_header(F.f, &h, true)) return e;
    *n = h.n;
    *r = h.r;
    *dtype = h.dtype;
    *dt = h.dt;
    return DMD_OK;
}

int32_t dmd_model_save(void* stream, const dmd_model* m, const char* path)
{
    if (!m || !path || !m->phi || !m->lam || !m->b || !m->sigma || !m->kind) return DMD_ERR_ARG;
    if (m->n < 1 || m->r < 1) return DMD_ERR_SHAPE;
    if (m->dtype != DMD_F32 && m->dtype != DMD_F64) return DMD_ERR_ARG;
    if (m->ldphi < m->r || !(m->dt > 0.0)) return DMD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int32_t r = m->r;
    const size_t esz = m->dtype == DMD_F64 ? 8 : 4;
    std::vector<double> lam(2 * (size_t)r), b(2 * (size_t)r), sigma((size_t)r);
    std::vector<int32_t> kind((size_t)r);
    HIPCHK_IO(hipMemcpyAsync(lam.data(), m->lam, lam.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK_IO(hipMemcpyAsync(b.data(), m->b, b.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK_IO(hipMemcpyAsync(sigma.data(), m->sigma, sigma.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK_IO(hipMemcpyAsync(kind.data(), m->kind, kind.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK_IO(hipStreamSynchronize(st));
    File F;
    F.f = fopen(path, "wb");
    if (!F.f) return DMD_ERR_IO;
    Header h{};
    memcpy(h.magic, MAGIC, 8);
    h.version = FORMAT_VERSION;
    h.header_bytes = HEADER_BYTES;
    h.n = m->n;
    h.r = r;
    h.dtype = m->dtype;
    h.dt = m->dt;
    h.payload_bytes = payload_bytes(m->n, r, m->dtype);
    h.abi = DMDMI_ABI_VERSION;
    if (fwrite(&h, 1, sizeof h, F.f) != sizeof h) return DMD_ERR_IO;   // hash written last
    Fnv fnv;
    auto put = [&](const void* p, size_t bytes) -> bool {
        fnv.add(p, bytes);
        return fwrite(p, 1, bytes, F.f) == bytes;
    };
    if (!put(lam.data(), lam.size() * 8) || !put(b.data(), b.size() * 8) || !put(sigma.data(), sigma.size() * 8) ||
        !put(kind.data(), kind.size() * 4))
        return DMD_ERR_IO;
    std::vector<char> rows((size_t)std::min<int64_t>(ROW_CHUNK, m->n) * r * esz);
    for (int64_t r0 = 0; r0 < m->n; r0 += ROW_CHUNK) {
        const int64_t nr = std::min<int64_t>(ROW_CHUNK, m->n - r0);
        const char* src = (const char*)m->phi + (size_t)r0 * m->ldphi * esz;
        HIPCHK_IO(hipMemcpy2DAsync(rows.data(), (size_t)r * esz, src, (size_t)m->ldphi * esz, (size_t)r * esz,
                                   (size_t)nr, hipMemcpyDeviceToHost, st));
        HIPCHK_IO(hipStreamSynchronize(st));
        if (!put(rows.data(), (size_t)nr * r * esz)) return DMD_ERR_IO;
    }
    h.hash = fnv.h;
    if (fseek(F.f, 0, SEEK_SET) != 0 || fwrite(&h, 1, sizeof h, F.f) != sizeof h) return DMD_ERR_IO;
    if (fflush(F.f) != 0) return DMD_ERR_IO;
    return DMD_OK;
}

int32_t dmd_model_load(void* stream, const char* path, dmd_model* m)
{
    if (!m || !path || !m->phi || !m->lam || !m->b || !m->sigma || !m->kind) return DMD_ERR_ARG;
    File F;
    F.f = fopen(path, "rb");
    if (!F.f) return DMD_ERR_IO;
    Header h;
    if (int32_t e = read_header(F.f, &h, true)) return e;
    if (m->n != h.n) return DMD_ERR_SHAPE;
    if (m->dtype != h.dtype) return DMD_ERR_ARG;
    if (m->ldphi < dmd_phi_ld(h.r) || m->ldphi % 32 != 0) return DMD_ERR_ARG;
    if (((uintptr_t)m->phi & 15u) != 0) return DMD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int32_t r = h.r;
    const size_t esz = h.dtype == DMD_F64 ? 8 : 4;
    std::vector<double> lam(2 * (size_t)r), b(2 * (size_t)r), sigma((size_t)r);
    std::vector<int32_t> kind((size_t)r);
    if (fread(lam.data(), 8, lam.size(), F.f) != lam.size() || fread(b.data(), 8, b.size(), F.f) != b.size() ||
        fread(sigma.data(), 8, sigma.size(), F.f) != sigma.size() || fread(kind.data(), 4, kind.size(), F.f) != kind.size())
        return DMD_ERR_IO;
    for (int32_t i = 0; i < r; ++i)
        if (kind[i] < 0 || kind[i] > 2) return DMD_ERR_IO;
    // rows of Phi staged with their zero padding columns, ROW_CHUNK rows at a time
    const int64_t ld = m->ldphi;
    std::vector<char> rows((size_t)std::min<int64_t>(ROW_CHUNK, h.n) * r * esz);
    std::vector<char> padded((size_t)std::min<int64_t>(ROW_CHUNK, h.n) * ld * esz, 0);
    for (int64_t r0 = 0; r0 < h.n; r0 += ROW_CHUNK) {
        const int64_t nr = std::min<int64_t>(ROW_CHUNK, h.n - r0);
        if (fread(rows.data(), 1, (size_t)nr * r * esz, F.f) != (size_t)nr * r * esz) return DMD_ERR_IO;
        HIPCHK_IO(hipStreamSynchronize(st));   // the previous chunk's copy has left `padded`
        for (int64_t i = 0; i < nr; ++i) memcpy(&padded[(size_t)i * ld * esz], &rows[(size_t)i * r * esz], (size_t)r * esz);
        char* dst = (char*)m->phi + (size_t)r0 * ld * esz;
        HIPCHK_IO(hipMemcpyAsync(dst, padded.data(), (size_t)nr * ld * esz, hipMemcpyHostToDevice, st));
    }
    HIPCHK_IO(hipMemcpyAsync(m->lam, lam.data(), lam.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK_IO(hipMemcpyAsync(m->b, b.data(), b.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK_IO(hipMemcpyAsync(m->sigma, sigma.data(), sigma.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK_IO(hipMemcpyAsync(m->kind, kind.data(), kind.size() * 4, hipMemcpyHostToDevice, st));
    if (m->info) {
        const int32_t zeros[DMD_INFO_WORDS] = {0};
        HIPCHK_IO(hipMemcpyAsync(m->info, zeros, sizeof zeros, hipMemcpyHostToDevice, st));
    }
    HIPCHK_IO(hipStreamSynchronize(st));   // host staging buffers end with this call
    m->r = r;
    m->dt = h.dt;
    return DMD_OK;
}

}  // extern "C"
