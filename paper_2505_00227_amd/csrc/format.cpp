// Container format (serialization, Sec. 5.1) and CRC-32.
//
// Little-endian throughout.
//   header (56 B): u32 magic 0x3152444D ("MDR1") | u8 version=1 | u8 dtype | u8 B | u8 m
//                  | u32 nlevels | u32 t_cr_milli | u64 t_s | u32 huf_chunk | u32 huf_lmax
//                  | i32 force_method | u32 0 | u64 blob bytes | u32 crc32(bytes 0..47) | u32 0
//   per level:     u64 n | i32 e | u32 nstreams=1+B | f64 min | f64 max | f64 max|x|
//                  | f64 E[B+1] | nstreams x {u8 method, u8[3] 0, u32 crc32, u64 bytes}
//                  | u32 crc32(record so far) | u32 0
//                  | payloads in table order, each zero padded to a multiple of 8 bytes
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "api_internal.hpp"

namespace mdr {

// ---- CRC-32 (reflected polynomial 0xEDB88320), eight table lookups per 8 bytes
namespace {
struct CrcTables {
    uint32_t t[8][256];
    CrcTables()
    {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1u) ? (c >> 1) ^ 0xEDB88320u : (c >> 1);
            t[0][i] = c;
        }
        for (int s = 1; s < 8; ++s)
            for (uint32_t i = 0; i < 256; ++i) t[s][i] = (t[s - 1][i] >> 8) ^ t[0][t[s - 1][i] & 0xFFu];
    }
};
const CrcTables& crc_tables()
{
    static const CrcTables tables;
    return tables;
}
}  // namespace

uint32_t crc32(const uint8_t* p, uint64_t n)
{
    const auto& T = crc_tables().t;
    uint32_t c = 0xFFFFFFFFu;
    while (n >= 8) {
        uint32_t a, b;
        std::memcpy(&a, p, 4);
        std::memcpy(&b, p + 4, 4);
        a ^= c;
        c = T[7][a & 0xFF] ^ T[6][(a >> 8) & 0xFF] ^ T[5][(a >> 16) & 0xFF] ^ T[4][a >> 24] ^
            T[3][b & 0xFF] ^ T[2][(b >> 8) & 0xFF] ^ T[1][(b >> 16) & 0xFF] ^ T[0][b >> 24];
        p += 8;
        n -= 8;
    }
    while (n--) c = (c >> 8) ^ T[0][(c ^ *p++) & 0xFFu];
    return c ^ 0xFFFFFFFFu;
}

namespace {
constexpr uint32_t kMagic = 0x3152444Du;
constexpr uint64_t kHeader = 56;

uint64_t pad8(uint64_t v) { return (v + 7) & ~(uint64_t)7; }

template <typename T>
void put(uint8_t* p, T v)
{
    std::memcpy(p, &v, sizeof(T));
}
template <typename T>
T get(const uint8_t* p)
{
    T v;
    std::memcpy(&v, p, sizeof(T));
    return v;
}

uint64_t record_bytes(uint32_t B) { return 16 + 24 + 8ull * (B + 1) + 16ull * (1 + B) + 8; }

uint64_t blob_size(const mdr_refactored* r)
{
    uint64_t t = kHeader;
    for (const LevelRec& L : r->levels) {
        t += record_bytes(r->B);
        for (uint32_t s = 0; s <= r->B; ++s)
            if (L.units[s].method != MDR_PLACEHOLDER) t += pad8(L.units[s].bytes);
    }
    return t;
}

mdr_status corrupt(const std::string& what) { return fail(MDR_ERR_CORRUPT_STREAM, what); }

uint64_t S_of(const mdr_refactored* r, const LevelRec& L, uint32_t slot)
{
    uint32_t r0, r1;
    slot_rows(slot, r->B, r->m, r0, r1);
    return 4ull * (r1 - r0) * L.nbd;
}

// structural checks of one payload (host bytes) so that decoding stays in bounds
mdr_status check_payload(const mdr_refactored* r, const LevelRec& L, uint32_t slot,
                         const uint8_t* p, uint64_t bytes, UnitRec& u)
{
    const uint64_t S = S_of(r, L, slot);
    u.S = S;
    if (u.method == MDR_DC) {
        if (bytes != S) return corrupt("direct-copy payload size does not match its planes");
        return MDR_OK;
    }
    if (u.method == MDR_RLE) {
        if (bytes < 8) return corrupt("RLE payload too short");
        uint64_t nr = get<uint32_t>(p);
        if (get<uint32_t>(p + 4) != 4 * r->G) return corrupt("RLE word width mismatch");
        if (bytes != 8 + nr * (4ull * r->G + 4)) return corrupt("RLE payload size mismatch");
        const uint64_t nwords = S / 4 / r->G;
        uint64_t total = 0;
        const uint8_t* lens = p + 8 + 4ull * r->G * nr;
        for (uint64_t i = 0; i < nr; ++i) {
            uint32_t len = get<uint32_t>(lens + 4 * i);
            if (len == 0) return corrupt("RLE run of length 0");
            total += len;
        }
        if (total != nwords) return corrupt("RLE runs do not cover the group");
        u.nruns = nr;
        return MDR_OK;
    }
    if (u.method == MDR_HUF) {
        const uint32_t chunk = r->prm.huf_chunk;
        const uint64_t nc = (S + chunk - 1) / chunk;
        if (bytes < 8 + 256 + 4 * (nc + 1)) return corrupt("Huffman payload too short");
        if (get<uint64_t>(p) != S) return corrupt("Huffman symbol count mismatch");
        uint32_t maxlen = 0;
        for (int s = 0; s < 256; ++s) {
            uint32_t l = p[8 + s];
            if (l > r->prm.huf_lmax) return corrupt("Huffman code longer than the limit");
            maxlen = l > maxlen ? l : maxlen;
        }
        const uint8_t* off = p + 8 + 256;
        const uint64_t words = (bytes - (8 + 256 + 4 * (nc + 1))) / 4;
        if (8 + 256 + 4 * (nc + 1) + 4 * words != bytes) return corrupt("Huffman payload not word aligned");
        uint32_t prev = 0;
        for (uint64_t c = 0; c <= nc; ++c) {
            uint32_t o = get<uint32_t>(off + 4 * c);
            if (o < prev || o > words) return corrupt("Huffman chunk offsets out of range");
            prev = o;
        }
        if (get<uint32_t>(off) != 0 || prev != words) return corrupt("Huffman chunk offsets inconsistent");
        u.nchunks = (uint32_t)nc;
        u.maxlen = maxlen;
        return MDR_OK;
    }
    return corrupt("unknown lossless method");
}
}  // namespace

}  // namespace mdr

using namespace mdr;

extern "C" {

mdr_status mdr_serialize(const mdr_refactored* r, void* host, uint64_t cap, uint64_t* used)
{
    set_error("");
    if (!r || !used) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    const uint64_t total = blob_size(r);
    *used = total;
    if (cap == 0) return MDR_OK;
    if (!host) return fail(MDR_ERR_INVALID_ARG, "host is NULL");
    if (cap < total) return fail(MDR_ERR_INVALID_ARG, "cap is smaller than the serialized size");
    hipError_t he = hipSetDevice(r->ctx->device);
    if (he != hipSuccess) return hip_fail(he, "hipSetDevice");
    he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(he, "hipDeviceSynchronize");
    uint8_t* out = static_cast<uint8_t*>(host);
    std::memset(out, 0, total);
    const uint32_t B = r->B;
    put<uint32_t>(out, kMagic);
    out[4] = 1;
    out[5] = (uint8_t)r->dtype;
    out[6] = (uint8_t)B;
    out[7] = (uint8_t)r->m;
    put<uint32_t>(out + 8, (uint32_t)r->levels.size());
    put<uint32_t>(out + 12, r->prm.t_cr_milli);
    put<uint64_t>(out + 16, r->prm.t_s_bytes);
    put<uint32_t>(out + 24, r->prm.huf_chunk);
    put<uint32_t>(out + 28, r->prm.huf_lmax);
    put<int32_t>(out + 32, r->prm.force_method);
    put<uint64_t>(out + 40, total);
    put<uint32_t>(out + 48, crc32(out, 48));
    uint64_t pos = kHeader;
    for (const LevelRec& L : r->levels) {
        const uint64_t rec = pos;
        put<uint64_t>(out + pos, L.n);
        put<int32_t>(out + pos + 8, L.e);
        put<uint32_t>(out + pos + 12, 1 + B);
        put<double>(out + pos + 16, L.vmin);
        put<double>(out + pos + 24, L.vmax);
        put<double>(out + pos + 32, L.vmaxabs);
        pos += 40;
        for (uint32_t k = 0; k <= B; ++k, pos += 8) put<double>(out + pos, L.E[k]);
        const uint64_t table = pos;
        pos += 16ull * (1 + B) + 8;
        // payloads first (their CRCs go into the table)
        for (uint32_t s = 0; s <= B; ++s) {
            const UnitRec& u = L.units[s];
            uint8_t* ent = out + table + 16ull * s;
            ent[0] = (uint8_t)u.method;
            uint64_t nb = u.method == MDR_PLACEHOLDER ? 0 : u.bytes;
            put<uint64_t>(ent + 8, nb);
            if (nb) {
                he = hipMemcpy(out + pos, u.dev, nb, hipMemcpyDeviceToHost);
                if (he != hipSuccess) return hip_fail(he, "hipMemcpy(payload)");
            }
            put<uint32_t>(ent + 4, crc32(out + pos, nb));
            if (u.method != MDR_PLACEHOLDER) pos += pad8(nb);
        }
        const uint64_t rec_end = table + 16ull * (1 + B);
        put<uint32_t>(out + rec_end, crc32(out + rec, rec_end - rec));
    }
    if (pos != total) return fail(MDR_ERR_HIP, "internal: serialized size mismatch");
    return MDR_OK;
}

mdr_status mdr_deserialize(mdr_context* ctx, const void* host, uint64_t bytes, mdr_refactored** out)
{
    set_error("");
    if (!out) return fail(MDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !host) return fail(MDR_ERR_INVALID_ARG, "NULL argument");
    const uint8_t* in = static_cast<const uint8_t*>(host);
    if (bytes < kHeader) return corrupt("blob shorter than its header");
    if (get<uint32_t>(in) != kMagic) return corrupt("bad magic");
    if (in[4] != 1) return corrupt("unknown container version");
    if (get<uint32_t>(in + 48) != crc32(in, 48)) return corrupt("header CRC mismatch");
    if (get<uint64_t>(in + 40) != bytes) return corrupt("blob size mismatch");
    auto R = std::make_unique<mdr_refactored>();
    R->ctx = ctx;
    if (in[5] > 1) return corrupt("bad dtype");
    R->dtype = (mdr_dtype)in[5];
    R->B = in[6];
    R->m = in[7];
    R->G = R->dtype == MDR_F64 ? 2 : 1;
    const uint32_t W = 32 * R->G, B = R->B, m = R->m;
    if (B < 1 || B > W || m < 1 || m > B) return corrupt("bad plane count or group size");
    const uint32_t nlevels = get<uint32_t>(in + 8);
    R->prm.group_planes = m;
    R->prm.t_cr_milli = get<uint32_t>(in + 12);
    R->prm.t_s_bytes = get<uint64_t>(in + 16);
    R->prm.huf_chunk = get<uint32_t>(in + 24);
    R->prm.huf_lmax = get<uint32_t>(in + 28);
    R->prm.force_method = get<int32_t>(in + 32);
    if (R->prm.huf_chunk < 256 || R->prm.huf_chunk > 4096 || (R->prm.huf_chunk & (R->prm.huf_chunk - 1)) ||
        R->prm.huf_lmax < 8 || R->prm.huf_lmax > (uint32_t)kLutBitsMax)
        return fail(MDR_ERR_UNSUPPORTED, "Huffman parameters not supported by this build");
    if (nlevels == 0 || nlevels > (bytes - kHeader) / record_bytes(B)) return corrupt("bad level count");
    R->levels.resize(nlevels);

    // ---- parse and validate everything on the host first
    struct Src {
        uint32_t level, slot;
        const uint8_t* p;
    };
    std::vector<Src> srcs;
    uint64_t pos = kHeader, rows_bytes = 0, pay_bytes = 0;
    for (uint32_t l = 0; l < nlevels; ++l) {
        LevelRec& L = R->levels[l];
        if (bytes - pos < record_bytes(B)) return corrupt("truncated level record");
        const uint64_t rec = pos;
        L.n = get<uint64_t>(in + pos);
        L.e = get<int32_t>(in + pos + 8);
        if (get<uint32_t>(in + pos + 12) != 1 + B) return corrupt("stream count mismatch");
        if (L.n > 0xFFFFFFFFull) return corrupt("level too large");
        L.nbd = R->G == 2 ? (uint32_t)(2 * ((L.n + 63) / 64)) : (uint32_t)((L.n + 31) / 32);
        L.vmin = get<double>(in + pos + 16);
        L.vmax = get<double>(in + pos + 24);
        L.vmaxabs = get<double>(in + pos + 32);
        pos += 40;
        L.E.resize(B + 1);
        for (uint32_t k = 0; k <= B; ++k, pos += 8) {
            L.E[k] = get<double>(in + pos);
            if (!(L.E[k] >= 0.0) || std::isinf(L.E[k])) return corrupt("bad error table");
        }
        const uint64_t table = pos;
        const uint64_t rec_end = table + 16ull * (1 + B);
        if (get<uint32_t>(in + rec_end) != crc32(in + rec, rec_end - rec)) return corrupt("level record CRC mismatch");
        pos = rec_end + 8;
        for (uint32_t s = 0; s <= B; ++s) {
            const uint8_t* ent = in + table + 16ull * s;
            UnitRec& u = L.units[s];
            u.method = ent[0];
            const uint64_t nb = get<uint64_t>(ent + 8);
            const bool leader = s == 0 || (s - 1) % m == 0;
            if (!leader) {
                if (u.method != MDR_PLACEHOLDER || nb != 0) return corrupt("bad placeholder slot");
                continue;
            }
            if (u.method > MDR_HUF) return corrupt("bad method in a leading slot");
            if (nb > bytes - pos) return corrupt("payload runs past the end of the blob");
            if (get<uint32_t>(ent + 4) != crc32(in + pos, nb)) return corrupt("payload CRC mismatch");
            u.bytes = nb;
            mdr_status st = check_payload(R.get(), L, s, in + pos, nb, u);
            if (st) return st;
            srcs.push_back({l, s, in + pos});
            if (u.method != MDR_DC) pay_bytes += (nb + 255) & ~255ull;
            pos += pad8(nb);
            if (pos > bytes) return corrupt("payload padding runs past the end of the blob");
        }
        rows_bytes += (4ull * (B + 1) * L.nbd + 255) & ~255ull;
    }
    if (pos != bytes) return corrupt("trailing bytes after the last level");

    // ---- upload: direct-copy payloads become plane rows, others go to the payload arena
    hipError_t he = hipSetDevice(ctx->device);
    if (he != hipSuccess) return hip_fail(he, "hipSetDevice");
    R->rows_arena = std::make_shared<PoolBuf>();
    R->payload_arena = std::make_shared<PoolBuf>();
    he = R->rows_arena->alloc(ctx->pool, rows_bytes);
    if (he != hipSuccess) return hip_fail(he, "hipMalloc(planes)");
    he = R->payload_arena->alloc(ctx->pool, pay_bytes + 256);  // padded for the Huffman decoder's block reads
    if (he != hipSuccess) return hip_fail(he, "hipMalloc(payloads)");
    uint8_t* rb = static_cast<uint8_t*>(R->rows_arena->p);
    for (uint32_t l = 0; l < nlevels; ++l) {
        R->levels[l].rows = reinterpret_cast<uint32_t*>(rb);
        rb += (4ull * (B + 1) * R->levels[l].nbd + 255) & ~255ull;
    }
    uint8_t* pb = static_cast<uint8_t*>(R->payload_arena->p);
    for (const Src& sr : srcs) {
        LevelRec& L = R->levels[sr.level];
        UnitRec& u = L.units[sr.slot];
        if (u.method == MDR_DC) {
            uint32_t r0, r1;
            slot_rows(sr.slot, B, m, r0, r1);
            u.dev = reinterpret_cast<uint8_t*>(L.rows + (uint64_t)r0 * L.nbd);
        } else {
            u.dev = pb;
            pb += (u.bytes + 255) & ~255ull;
        }
        if (u.bytes) {
            he = hipMemcpy(u.dev, sr.p, u.bytes, hipMemcpyHostToDevice);
            if (he != hipSuccess) return hip_fail(he, "hipMemcpy(payload)");
        }
    }
    *out = R.release();
    return MDR_OK;
}

}  // extern "C"
