/*
 * mdr_oracle.c -- plain CPU oracle for HP-MDR's bitplane + lossless path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  Nothing in the product library includes,
 * links or calls this file; the two implementations share no code.
 *
 * Style: every step is written as its definition, one value / one bit at a
 * time, in the order the paper states it.  Floating point is done in double
 * (every intermediate used here is exact, as argued at each step).  No
 * blocking, fusion or reordering beyond the definitions.
 *
 * Readings of passages that the paper leaves open are marked "reading:"; the
 * full list is kept with the design notes of the repository.
 *
 * Parity pins (tests/test_oracle_*.py) are named at each function.  Functions
 * whose behaviour is a format choice of this project (Huffman tie-breaks and
 * chunking, RLE layout, container layout) are pinned by round trips and
 * closed forms only: their exact bytes are "parity unpinned" against the
 * paper, which prints none.
 */
#include "mdr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* threads (the oracle's per-value loops may run on all host cores)          */
/* ------------------------------------------------------------------------ */
void orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    omp_set_num_threads(nthreads > 0 ? nthreads : 1);
#else
    (void)nthreads;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double value_at(const void* x, int dtype, uint64_t i)
{
    if (dtype == ORC_F32) return (double)((const float*)x)[i]; /* exact widening */
    return ((const double*)x)[i];
}

/* ------------------------------------------------------------------------ */
/* Sec. 3 / Alg. 1 step 1: level statistics and the alignment exponent        */
/* ------------------------------------------------------------------------ */
/*
 * e = the largest binary exponent over the nonzero values of the level, in
 * the frexp convention (|x| < 2^e and max|x| >= 2^(e-1)); e = 0 when every
 * value is zero.  Reading: "global maximum exponent" taken per level
 * (Alg. 1 works on one decomposed array) with the frexp convention, so that
 * the aligned magnitude fits in B bits.  Non-finite input is rejected.
 * min / max / max|x| are recorded for relative tolerances; a zero of either
 * sign is recorded as +0.0.
 * Pins: numpy.frexp of max|x|; brute force on tiny inputs; special cases.
 */
int orc_stats(const void* x, uint64_t n, int dtype, int32_t* e, double* vmin, double* vmax,
              double* vmaxabs)
{
    int have = 0;
    int emax = 0;
    double lo = 0.0, hi = 0.0, amax = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        double v = value_at(x, dtype, i);
        if (!isfinite(v)) return ORC_EINVAL;
        if (i == 0) {
            lo = v;
            hi = v;
        }
        if (v < lo) lo = v;
        if (v > hi) hi = v;
        if (fabs(v) > amax) amax = fabs(v);
        if (v != 0.0) {
            int ex = 0;
            frexp(v, &ex);
            if (!have || ex > emax) {
                emax = ex;
                have = 1;
            }
        }
    }
    *e = have ? emax : 0;
    *vmin = (lo == 0.0) ? 0.0 : lo;
    *vmax = (hi == 0.0) ? 0.0 : hi;
    *vmaxabs = amax;
    return ORC_OK;
}

/*
 * Alg. 1 step 1 (AlignExponent) as sign / magnitude fixed point:
 *   mag_i  = floor(|x_i| * 2^(B - e))   (an integer < 2^B)
 *   sign_i = sign bit of x_i            (-0.0 has sign 1)
 * Reading: truncation (the algorithm only extracts bits), separate sign plane.
 * Exactness: |x| * 2^(B-e) is a power-of-two scaling; it is exact unless the
 * result falls below the normal range, and then it is < 1 and floors to 0
 * either way.  The result is < 2^B <= 2^64, so the integer conversion is exact.
 * Pins: brute-force search for the largest m with m*2^(e-B) <= |x| (Fraction);
 * |x| = 2^(e-1) gives 2^(B-1); subnormal-only levels; -0.0.
 */
void orc_fixed_point(const void* x, uint64_t n, int dtype, int32_t e, uint32_t B, uint64_t* mag,
                     uint8_t* sign)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        double v = value_at(x, dtype, (uint64_t)i);
        double scaled = ldexp(fabs(v), (int)B - (int)e);
        mag[i] = (uint64_t)floor(scaled);
        sign[i] = signbit(v) ? 1 : 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 loop: bitplanes, most significant first                             */
/* ------------------------------------------------------------------------ */
/*
 * A plane holds one bit of every value of the level.  Reading of the storage
 * order (the paper's locality-block layout, Sec. 3.1): value i's bit is bit
 * (i mod W) of the W-bit little-endian word i / W, i.e. bit i of the plane's
 * byte string, least significant bit first.  Words beyond n are padded with
 * zero bits; a plane therefore has ceil(n / W) words.
 */
uint64_t orc_plane_bytes(uint64_t n, uint32_t W)
{
    return ((n + W - 1) / W) * (W / 8);
}

static void write_bitplane(uint8_t* dst, const uint8_t* bits, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i)
        if (bits[i]) dst[i / 8] |= (uint8_t)(1u << (i % 8));
}

/*
 * rows[0] = sign plane, rows[1 + p] = magnitude plane p, which holds bit
 * b = B-1-p (the loop of Alg. 1 runs b from B-1 down to 0 and flushes one
 * plane per b).
 * Pins: a pure-Python bit-string transcription on random inputs; invertibility
 * (reassembling the planes returns every magnitude); hand-computed fixture.
 */
void orc_bitplanes(const uint64_t* mag, const uint8_t* sign, uint64_t n, uint32_t B, uint32_t W,
                   uint8_t* rows)
{
    uint64_t pb = orc_plane_bytes(n, W);
    memset(rows, 0, (size_t)(pb * (B + 1)));
    uint8_t* bitplane = (uint8_t*)malloc(n ? (size_t)n : 1);
    for (uint64_t i = 0; i < n; ++i) bitplane[i] = sign[i];
    write_bitplane(rows, bitplane, n);
    uint32_t row = 1;
    for (int b = (int)B - 1; b >= 0; --b) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)n; ++i) bitplane[i] = (uint8_t)((mag[i] >> b) & 1u);
        write_bitplane(rows + (uint64_t)row * pb, bitplane, n);
        ++row;
    }
    free(bitplane);
}

/*
 * Sec. 3's encoding experiment: n 32-bit words into 32 bitplanes, plane p =
 * bit 31-p, plane-major, `words` 32-bit words per plane, values past n = 0.
 * interleaved = 0 (locality block, and the register-shuffling designs): bit t of
 * word j is value 32j + t.  interleaved = 1 (register block): the values of a
 * 2048-value region r are spread over 64 words, bit k of word 64r + l being
 * value 2048r + l + 64k.
 * Pins: single-bit inputs by hand; the block layout equals the magnitude rows
 * of orc_bitplanes; the interleaved layout is the block layout of the input
 * reordered region by region.
 */
void orc_abl_planes(int interleaved, const uint32_t* in, uint64_t n, uint32_t* planes, uint64_t words)
{
    memset(planes, 0, (size_t)(32 * words * 4));
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t word, bit;
        if (interleaved) {
            uint64_t r = i / 2048, o = i % 2048;
            word = 64 * r + o % 64;
            bit = o / 64;
        } else {
            word = i / 32;
            bit = i % 32;
        }
        for (int p = 0; p < 32; ++p)
            if ((in[i] >> (31 - p)) & 1u) planes[(uint64_t)p * words + word] |= 1u << bit;
    }
}

/* ------------------------------------------------------------------------ */
/* per-plane error table                                                      */
/* ------------------------------------------------------------------------ */
/* magnitude keeping only its top k of B bits (k planes retrieved) */
static uint64_t keep_top(uint64_t m, uint32_t B, uint32_t k)
{
    if (k == 0) return 0;
    uint32_t drop = B - k;
    if (drop == 0) return m;
    return m & ~((((uint64_t)1) << drop) - 1);
}

/*
 * E[k] = max_i ( |x_i| - |xhat_i^(k)| ),  k = 0..B, where xhat^(k) is the value
 * rebuilt from the sign and the top k planes:
 *   |xhat^(k)| = keep_top(mag, k) * 2^(e - B).
 * Reading: the paper only says that retrieval meets an error bound from the
 * planes it fetches; the table is MDR's L-infinity error after k planes.
 * Exactness: |xhat| is |x| truncated to a multiple of 2^(e-k), so it is a
 * subset of |x|'s significand bits (the integer conversion and the ldexp are
 * exact) and |x| - |xhat| is exact (Sterbenz, or |xhat| = 0).  Every E[k] is
 * therefore exactly representable in the input type.
 * Pins: Fraction brute force; E[0] = max|x|; E non-increasing; E[k] < 2^(e-k);
 * pointwise |x - xhat^(k)| <= E[k].
 */
void orc_error_table(const void* x, const uint64_t* mag, uint64_t n, int dtype, int32_t e,
                     uint32_t B, double* E)
{
    for (uint32_t k = 0; k <= B; ++k) {
        double worst = 0.0;
#pragma omp parallel for schedule(static) reduction(max : worst)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            double a = fabs(value_at(x, dtype, (uint64_t)i));
            double xhat = ldexp((double)keep_top(mag[i], B, k), (int)e - (int)B);
            double err = a - xhat;
            if (err > worst) worst = err;
        }
        E[k] = worst;
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1 Huffman coding of the merged planes (byte symbols)               */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t w;
    int sym;
} leaf_t;

static int leaf_cmp(const void* a, const void* b)
{
    const leaf_t* x = (const leaf_t*)a;
    const leaf_t* y = (const leaf_t*)b;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return x->sym - y->sym;
}

/*
 * Optimal code lengths by the two-queue Huffman construction.
 * Reading (format choices; the paper defers to a GPU Huffman coder):
 *  - leaves are the symbols with nonzero count, ordered by (count, symbol);
 *  - each merge takes the two lightest nodes, preferring the leaf queue on a
 *    weight tie; merged nodes are queued in creation order;
 *  - a single distinct symbol gets a phantom partner (the smallest other
 *    symbol) so both have length 1.
 * Fills the sorted leaves and their depths; returns the number of leaves.
 */
static int huffman_tree(const uint64_t* f, leaf_t* leaves, int* depth_of_leaf)
{
    int nl = 0;
    for (int s = 0; s < 256; ++s)
        if (f[s]) {
            leaves[nl].w = f[s];
            leaves[nl].sym = s;
            ++nl;
        }
    if (nl < 2) return nl;
    qsort(leaves, (size_t)nl, sizeof(leaf_t), leaf_cmp);

    uint64_t w[512];
    int parent[512];
    int depth[512];
    for (int i = 0; i < nl; ++i) w[i] = leaves[i].w;
    int q1 = 0;       /* next unused leaf */
    int q2 = nl;      /* next unused merged node */
    int next = nl;    /* next node index to create */
    while ((nl - q1) + (next - q2) > 1) {
        int pick[2];
        for (int t = 0; t < 2; ++t) {
            if (q1 < nl && (q2 == next || w[q1] <= w[q2]))
                pick[t] = q1++;
            else
                pick[t] = q2++;
        }
        w[next] = w[pick[0]] + w[pick[1]];
        parent[pick[0]] = next;
        parent[pick[1]] = next;
        ++next;
    }
    int root = next - 1;
    depth[root] = 0;
    for (int i = root - 1; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
    for (int i = 0; i < nl; ++i) depth_of_leaf[i] = depth[i];
    return nl;
}

/*
 * Code lengths limited to lmax.
 * Reading (length limit): when the tree is deeper than lmax, the number of
 * codes of each length, BITS[L], is adjusted as in ITU-T T.81 Annex K
 * (Adjust_BITS): while some length i > lmax has codes, take two codes of
 * length i, give one of them length i-1, and split the longest code shorter
 * than i-1 (length j) into two codes of length j+1.  Each move keeps the code
 * count and the Kraft sum (= 1).  The lengths are then handed out again in the
 * leaves' (count, symbol) order: the heaviest leaves get the shortest lengths.
 * Trees within the limit keep their own lengths.
 * Pins: Kraft equality; sum f*L equals the textbook heap Huffman cost when the
 * limit is not hit; brute-force optimal prefix code for <= 6 symbols;
 * Fibonacci counts force the limit; limited lengths never increase with count.
 */
int orc_huffman_lengths(const uint64_t* freq, uint32_t lmax, uint8_t* len)
{
    if (lmax < 8 || lmax > 24) return ORC_EUNSUP;
    leaf_t leaves[256];
    int depth[256];
    memset(len, 0, 256);
    int nl = huffman_tree(freq, leaves, depth);
    if (nl == 0) return ORC_OK;
    if (nl == 1) {
        int s0 = leaves[0].sym;
        len[s0] = 1;
        len[s0 == 0 ? 1 : 0] = 1;
        return ORC_OK;
    }
    int maxlen = 0;
    for (int i = 0; i < nl; ++i) maxlen = depth[i] > maxlen ? depth[i] : maxlen;
    if (maxlen <= (int)lmax) {
        for (int i = 0; i < nl; ++i) len[leaves[i].sym] = (uint8_t)depth[i];
        return ORC_OK;
    }
    int bits[256 + 1];
    memset(bits, 0, sizeof(bits));
    for (int i = 0; i < nl; ++i) bits[depth[i]]++;
    for (int i = maxlen; i > (int)lmax; --i) {
        while (bits[i] > 0) {
            int j = i - 2;
            while (bits[j] == 0) --j;
            bits[i] -= 2;
            bits[i - 1] += 1;
            bits[j + 1] += 2;
            bits[j] -= 1;
        }
    }
    /* heaviest leaf (last in the sorted order) gets the shortest length */
    int L = 1, used = 0;
    for (int i = nl - 1; i >= 0; --i) {
        while (used == bits[L]) {
            ++L;
            used = 0;
        }
        len[leaves[i].sym] = (uint8_t)L;
        ++used;
    }
    return ORC_OK;
}

/* canonical codes: symbols ordered by (length, symbol); consecutive codes */
void orc_huffman_codes(const uint8_t* len, uint32_t* code)
{
    uint32_t c = 0;
    int prev = 0;
    int first = 1;
    memset(code, 0, 256 * sizeof(uint32_t));
    for (int L = 1; L <= 32; ++L)
        for (int s = 0; s < 256; ++s)
            if (len[s] == L) {
                if (first) {
                    c = 0;
                    first = 0;
                } else {
                    c = (c + 1) << (L - prev);
                }
                code[s] = c;
                prev = L;
            }
}

static uint64_t n_chunks(uint64_t S, uint32_t chunk)
{
    return (S + chunk - 1) / chunk;
}

/*
 * Huffman size estimate of Alg. 2 (Sec. 4.2, Huffman CR estimation):
 *   ceil(sum_s f_s * L_s / 8) bytes of code bits, plus the constant payload
 *   header: u64 symbol count + 256 code lengths + (nchunks+1) u32 offsets.
 * (The real payload is a little larger: each chunk is padded to a u32 word.)
 */
uint64_t orc_huffman_estimate(const uint64_t* freq, const uint8_t* len, uint64_t S, uint32_t chunk)
{
    uint64_t bits = 0;
    for (int s = 0; s < 256; ++s) bits += freq[s] * (uint64_t)len[s];
    return (bits + 7) / 8 + 8 + 256 + 4 * (n_chunks(S, chunk) + 1);
}

static void byte_histogram(const uint8_t* g, uint64_t S, uint64_t* freq)
{
    memset(freq, 0, 256 * sizeof(uint64_t));
    for (uint64_t i = 0; i < S; ++i) freq[g[i]]++;
}

static void put_u32(uint8_t* p, uint32_t v)
{
    for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t* p, uint64_t v)
{
    for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static uint32_t get_u32(const uint8_t* p)
{
    uint32_t v = 0;
    for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i);
    return v;
}
static uint64_t get_u64(const uint8_t* p)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

/* bits of one chunk: sum of code lengths of its symbols */
static uint64_t chunk_bits(const uint8_t* g, uint64_t S, uint64_t c, uint32_t chunk,
                           const uint8_t* len)
{
    uint64_t lo = c * chunk, hi = lo + chunk;
    if (hi > S) hi = S;
    uint64_t bits = 0;
    for (uint64_t i = lo; i < hi; ++i) bits += len[g[i]];
    return bits;
}

/*
 * Huffman payload (format of this project):
 *   u64 nsym | u8 len[256] | u32 off[nchunks+1] | u32 words[off[nchunks]]
 * Chunk c codes symbols [c*chunk, min(S,(c+1)*chunk)) starting at word off[c];
 * code bits are packed most significant bit first (first bit -> bit 31 of the
 * first word); the chunk's last word is zero padded.
 */
uint64_t orc_huffman_encoded_size(const uint8_t* g, uint64_t S, uint32_t chunk, uint32_t lmax)
{
    uint64_t freq[256];
    uint8_t len[256];
    byte_histogram(g, S, freq);
    if (orc_huffman_lengths(freq, lmax, len) != ORC_OK) return 0;
    uint64_t nc = n_chunks(S, chunk), words = 0;
    for (uint64_t c = 0; c < nc; ++c) words += (chunk_bits(g, S, c, chunk, len) + 31) / 32;
    return 8 + 256 + 4 * (nc + 1) + 4 * words;
}

int orc_huffman_encode(const uint8_t* g, uint64_t S, uint32_t chunk, uint32_t lmax, uint8_t* out,
                       uint64_t cap, uint64_t* used)
{
    if (chunk == 0) return ORC_EINVAL;
    uint64_t freq[256];
    uint8_t len[256];
    uint32_t code[256];
    byte_histogram(g, S, freq);
    int st = orc_huffman_lengths(freq, lmax, len);
    if (st != ORC_OK) return st;
    orc_huffman_codes(len, code);
    uint64_t nc = n_chunks(S, chunk);
    uint64_t need = orc_huffman_encoded_size(g, S, chunk, lmax);
    *used = need;
    if (cap < need) return ORC_ENOMEM;
    memset(out, 0, (size_t)need);
    put_u64(out, S);
    memcpy(out + 8, len, 256);
    uint8_t* offp = out + 8 + 256;
    uint8_t* words = offp + 4 * (nc + 1);
    uint64_t w = 0;
    for (uint64_t c = 0; c < nc; ++c) {
        put_u32(offp + 4 * c, (uint32_t)w);
        uint64_t lo = c * chunk, hi = lo + chunk;
        if (hi > S) hi = S;
        uint64_t bitpos = 0; /* within this chunk */
        for (uint64_t i = lo; i < hi; ++i) {
            uint32_t L = len[g[i]], cd = code[g[i]];
            for (int j = (int)L - 1; j >= 0; --j) {
                uint32_t bit = (cd >> j) & 1u;
                uint64_t word = w + bitpos / 32;
                uint32_t cur = get_u32(words + 4 * word);
                cur |= bit << (31 - (bitpos % 32));
                put_u32(words + 4 * word, cur);
                ++bitpos;
            }
        }
        w += (bitpos + 31) / 32;
    }
    put_u32(offp + 4 * nc, (uint32_t)w);
    return ORC_OK;
}

/* canonical decoding, one bit at a time */
int orc_huffman_decode(const uint8_t* p, uint64_t bytes, uint32_t chunk, uint8_t* g, uint64_t S)
{
    if (bytes < 8 + 256 + 4 || chunk == 0) return ORC_ECORRUPT;
    if (get_u64(p) != S) return ORC_ECORRUPT;
    const uint8_t* len = p + 8;
    uint64_t nc = n_chunks(S, chunk);
    if (bytes < 8 + 256 + 4 * (nc + 1)) return ORC_ECORRUPT;
    const uint8_t* offp = p + 8 + 256;
    const uint8_t* words = offp + 4 * (nc + 1);
    uint64_t nwords = (bytes - (8 + 256 + 4 * (nc + 1))) / 4;
    if (get_u32(offp + 4 * nc) != nwords) return ORC_ECORRUPT;

    /* per-length tables of the canonical code */
    int count[33] = {0};
    for (int s = 0; s < 256; ++s) {
        if (len[s] > 32) return ORC_ECORRUPT;
        if (len[s]) count[len[s]]++;
    }
    int sorted[256], pos = 0;
    int offset[33];
    uint64_t first[33];
    uint64_t c = 0;
    for (int L = 1; L <= 32; ++L) {
        offset[L] = pos;
        first[L] = c;
        for (int s = 0; s < 256; ++s)
            if (len[s] == L) sorted[pos++] = s;
        c = (c + (uint64_t)count[L]) << 1;
    }
    for (uint64_t ch = 0; ch < nc; ++ch) {
        uint64_t lo = ch * chunk, hi = lo + chunk;
        if (hi > S) hi = S;
        uint64_t w0 = get_u32(offp + 4 * ch), w1 = get_u32(offp + 4 * (ch + 1));
        if (w1 < w0 || w1 > nwords) return ORC_ECORRUPT;
        uint64_t bitpos = 0, nbits = (w1 - w0) * 32;
        for (uint64_t i = lo; i < hi; ++i) {
            uint64_t code = 0;
            int L = 0;
            for (;;) {
                if (bitpos >= nbits || L >= 32) return ORC_ECORRUPT;
                uint32_t word = get_u32(words + 4 * (w0 + bitpos / 32));
                code = (code << 1) | ((word >> (31 - (bitpos % 32))) & 1u);
                ++bitpos;
                ++L;
                if (count[L] && code - first[L] < (uint64_t)count[L] && code >= first[L]) {
                    g[i] = (uint8_t)sorted[offset[L] + (int)(code - first[L])];
                    break;
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1 run-length encoding of W-bit plane words                          */
/* ------------------------------------------------------------------------ */
static int word_eq(const uint8_t* g, uint64_t i, uint64_t j, uint32_t wb)
{
    return memcmp(g + i * wb, g + j * wb, wb) == 0;
}

/* number of maximal runs of equal W-bit words (Sec. 4.2, RLE CR estimation) */
uint64_t orc_rle_runs(const uint8_t* g, uint64_t S, uint32_t wbytes)
{
    uint64_t nw = S / wbytes, runs = 0;
    for (uint64_t i = 0; i < nw; ++i)
        if (i == 0 || !word_eq(g, i, i - 1, wbytes)) ++runs;
    return runs;
}

/*
 * RLE payload (format of this project; symbol = one W-bit plane word, run
 * length = u32):  u32 nruns | u32 wbytes | symbols[nruns] | u32 lengths[nruns].
 * The estimate of Alg. 2 is the exact payload size: a fixed cost per run for
 * the symbol plus the run-length field.
 */
uint64_t orc_rle_estimate(uint64_t nruns, uint32_t wbytes)
{
    return 8 + nruns * ((uint64_t)wbytes + 4);
}

int orc_rle_encode(const uint8_t* g, uint64_t S, uint32_t wbytes, uint8_t* out, uint64_t cap,
                   uint64_t* used)
{
    if (wbytes == 0 || S % wbytes) return ORC_EINVAL;
    uint64_t nr = orc_rle_runs(g, S, wbytes);
    uint64_t need = orc_rle_estimate(nr, wbytes);
    *used = need;
    if (cap < need) return ORC_ENOMEM;
    put_u32(out, (uint32_t)nr);
    put_u32(out + 4, wbytes);
    uint8_t* sym = out + 8;
    uint8_t* lens = sym + nr * wbytes;
    uint64_t nw = S / wbytes, r = 0, runlen = 0;
    for (uint64_t i = 0; i < nw; ++i) {
        if (i == 0 || !word_eq(g, i, i - 1, wbytes)) {
            if (i > 0) put_u32(lens + 4 * (r - 1), (uint32_t)runlen);
            memcpy(sym + r * wbytes, g + i * wbytes, wbytes);
            ++r;
            runlen = 0;
        }
        ++runlen;
    }
    if (r > 0) put_u32(lens + 4 * (r - 1), (uint32_t)runlen);
    return ORC_OK;
}

int orc_rle_decode(const uint8_t* p, uint64_t bytes, uint32_t wbytes, uint8_t* g, uint64_t S)
{
    if (bytes < 8) return ORC_ECORRUPT;
    uint64_t nr = get_u32(p);
    if (get_u32(p + 4) != wbytes) return ORC_ECORRUPT;
    if (bytes != orc_rle_estimate(nr, wbytes)) return ORC_ECORRUPT;
    const uint8_t* sym = p + 8;
    const uint8_t* lens = sym + nr * wbytes;
    uint64_t nw = S / wbytes, w = 0;
    for (uint64_t r = 0; r < nr; ++r) {
        uint64_t L = get_u32(lens + 4 * r);
        if (L == 0 || w + L > nw) return ORC_ECORRUPT;
        for (uint64_t j = 0; j < L; ++j) memcpy(g + (w + j) * wbytes, sym + r * wbytes, wbytes);
        w += L;
    }
    return w == nw ? ORC_OK : ORC_ECORRUPT;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2 Alg. 2: hybrid selection for one unit of S bytes                 */
/* ------------------------------------------------------------------------ */
/*
 * if S > T_s:  Huffman if r_H > T_cr, else RLE if r_R > T_cr, else DC;
 * otherwise DC.  r_X = S / est_X; the comparison is done in integers:
 * r_X > T_cr  <=>  1000*S > t_cr_milli * est_X.
 * Reading: the literal order of Alg. 2 (Huffman tested first).
 * Pins: a literal decision table on hand-built groups.
 */
int orc_select(uint64_t S, uint64_t est_huf, uint64_t est_rle, const orc_params* prm)
{
    if (prm->force_method >= 0) return prm->force_method;
    if (S > prm->t_s) {
        if (1000 * S > (uint64_t)prm->t_cr_milli * est_huf) return ORC_HUF;
        if (1000 * S > (uint64_t)prm->t_cr_milli * est_rle) return ORC_RLE;
        return ORC_DC;
    }
    return ORC_DC;
}

/* ------------------------------------------------------------------------ */
/* CRC-32 (IEEE 802.3, reflected, polynomial 0xEDB88320), bit at a time       */
/* ------------------------------------------------------------------------ */
uint32_t orc_crc32(const uint8_t* p, uint64_t n)
{
    uint32_t c = 0xFFFFFFFFu;
    for (uint64_t i = 0; i < n; ++i) {
        c ^= p[i];
        for (int k = 0; k < 8; ++k) c = (c & 1u) ? (c >> 1) ^ 0xEDB88320u : (c >> 1);
    }
    return c ^ 0xFFFFFFFFu;
}

/* ------------------------------------------------------------------------ */
/* one level, end to end                                                      */
/* ------------------------------------------------------------------------ */
struct orc_level {
    int dtype;
    uint32_t B, W, m;
    uint64_t n, plane_bytes;
    int32_t e;
    double vmin, vmax, vmaxabs;
    double E[65];
    orc_params prm;
    uint8_t* rows; /* (B+1) planes; row 0 = sign */
    int32_t method[65];
    uint64_t bytes[65];
    uint8_t* data[65];
    uint64_t est_huf[65], est_rle[65];
};

/*
 * Units of Alg. 2 (reading of "merge B[i..i+m-1]" with i stepping by m):
 *   unit 0  = the sign plane alone;
 *   group g = magnitude planes [g*m, min(B, (g+1)*m)), concatenated.
 * The group's payload sits at its leading plane; the other planes of the
 * group are placeholders of 0 bytes (Alg. 2, placeholder slots).
 * Table index: 0 = sign, 1 + p = plane p.
 */
static int encode_unit(orc_level* L, int slot, const uint8_t* g, uint64_t S)
{
    uint64_t freq[256];
    uint8_t len[256];
    uint32_t wb = L->W / 8;
    byte_histogram(g, S, freq);
    int st = orc_huffman_lengths(freq, L->prm.huf_lmax, len);
    if (st != ORC_OK) return st;
    L->est_huf[slot] = orc_huffman_estimate(freq, len, S, L->prm.huf_chunk);
    L->est_rle[slot] = orc_rle_estimate(orc_rle_runs(g, S, wb), wb);
    int meth = orc_select(S, L->est_huf[slot], L->est_rle[slot], &L->prm);
    L->method[slot] = meth;
    uint64_t used = 0;
    if (meth == ORC_DC) {
        L->data[slot] = (uint8_t*)malloc(S ? (size_t)S : 1);
        memcpy(L->data[slot], g, (size_t)S);
        used = S;
    } else if (meth == ORC_RLE) {
        uint64_t cap = orc_rle_estimate(orc_rle_runs(g, S, wb), wb);
        L->data[slot] = (uint8_t*)malloc((size_t)cap);
        st = orc_rle_encode(g, S, wb, L->data[slot], cap, &used);
    } else if (meth == ORC_HUF) {
        uint64_t cap = orc_huffman_encoded_size(g, S, L->prm.huf_chunk, L->prm.huf_lmax);
        L->data[slot] = (uint8_t*)malloc((size_t)cap);
        st = orc_huffman_encode(g, S, L->prm.huf_chunk, L->prm.huf_lmax, L->data[slot], cap, &used);
    } else {
        return ORC_EINVAL;
    }
    L->bytes[slot] = used;
    return st;
}

void orc_level_free(orc_level* L)
{
    if (!L) return;
    free(L->rows);
    for (int i = 0; i < 65; ++i) free(L->data[i]);
    free(L);
}

int orc_refactor_level(const void* x, uint64_t n, int dtype, uint32_t B, const orc_params* prm,
                       orc_level** out)
{
    *out = NULL;
    if (dtype != ORC_F32 && dtype != ORC_F64) return ORC_EINVAL;
    uint32_t W = dtype == ORC_F32 ? 32 : 64;
    if (B < 1 || B > W) return ORC_EUNSUP;
    if (prm->group_planes < 1 || prm->huf_chunk < 1) return ORC_EINVAL;
    if (prm->force_method > ORC_HUF) return ORC_EINVAL;
    orc_level* L = (orc_level*)calloc(1, sizeof(orc_level));
    L->dtype = dtype;
    L->B = B;
    L->W = W;
    L->m = prm->group_planes < B ? prm->group_planes : B;
    L->n = n;
    L->prm = *prm;
    int st = orc_stats(x, n, dtype, &L->e, &L->vmin, &L->vmax, &L->vmaxabs);
    if (st != ORC_OK) {
        orc_level_free(L);
        return st;
    }
    uint64_t* mag = (uint64_t*)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    uint8_t* sign = (uint8_t*)malloc((size_t)(n ? n : 1));
    orc_fixed_point(x, n, dtype, L->e, B, mag, sign);
    L->plane_bytes = orc_plane_bytes(n, W);
    L->rows = (uint8_t*)malloc((size_t)(L->plane_bytes * (B + 1) + 1));
    orc_bitplanes(mag, sign, n, B, W, L->rows);
    orc_error_table(x, mag, n, dtype, L->e, B, L->E);
    free(mag);
    free(sign);

    for (int i = 0; i < 65; ++i) L->method[i] = ORC_PLACEHOLDER;
    st = encode_unit(L, 0, L->rows, L->plane_bytes);
    for (uint32_t p0 = 0; st == ORC_OK && p0 < B; p0 += L->m) {
        uint32_t p1 = p0 + L->m < B ? p0 + L->m : B;
        st = encode_unit(L, 1 + (int)p0, L->rows + (uint64_t)(1 + p0) * L->plane_bytes,
                         (uint64_t)(p1 - p0) * L->plane_bytes);
    }
    if (st != ORC_OK) {
        orc_level_free(L);
        return st;
    }
    *out = L;
    return ORC_OK;
}

int orc_level_info(const orc_level* L, uint64_t* n, int32_t* e, double* vmin, double* vmax,
                   double* vmaxabs, double* E)
{
    *n = L->n;
    *e = L->e;
    *vmin = L->vmin;
    *vmax = L->vmax;
    *vmaxabs = L->vmaxabs;
    for (uint32_t k = 0; k <= L->B; ++k) E[k] = L->E[k];
    return ORC_OK;
}

int orc_level_stream(const orc_level* L, int32_t stream, int32_t* method, uint64_t* bytes,
                     const uint8_t** data, uint64_t* est_huf, uint64_t* est_rle)
{
    if (stream < -1 || stream >= (int32_t)L->B) return ORC_EINVAL;
    int slot = stream + 1;
    *method = L->method[slot];
    *bytes = L->method[slot] == ORC_PLACEHOLDER ? 0 : L->bytes[slot];
    *data = L->data[slot];
    *est_huf = L->est_huf[slot];
    *est_rle = L->est_rle[slot];
    return ORC_OK;
}

const uint8_t* orc_level_rows(const orc_level* L, uint64_t* plane_bytes)
{
    *plane_bytes = L->plane_bytes;
    return L->rows;
}

/* decode the unit in table slot `slot` back into its concatenated planes */
static int decode_unit(const orc_level* L, int slot, uint8_t* g, uint64_t S)
{
    switch (L->method[slot]) {
    case ORC_DC:
        if (L->bytes[slot] != S) return ORC_ECORRUPT;
        memcpy(g, L->data[slot], (size_t)S);
        return ORC_OK;
    case ORC_RLE: return orc_rle_decode(L->data[slot], L->bytes[slot], L->W / 8, g, S);
    case ORC_HUF: return orc_huffman_decode(L->data[slot], L->bytes[slot], L->prm.huf_chunk, g, S);
    default: return ORC_ECORRUPT;
    }
}

/*
 * Retrieval of one level from its first k magnitude planes (inverse of Alg. 1):
 * decode the sign unit and every group that starts below plane k, rebuild
 *   mag_i = sum over planes p < k of bit_i(plane p) << (B-1-p)
 * and x_i = (-1)^sign_i * mag_i * 2^(e-B) (exact, see orc_error_table).
 * With k = 0 nothing is fetched and every value is +0.0.
 * Pins: round trip with all planes on values that are multiples of 2^(e-B);
 * the bound |x - xhat| <= E[k] <= 2^(e-k).
 */
int orc_reconstruct(const orc_level* L, uint32_t k, void* out)
{
    if (k > L->B) return ORC_EINVAL;
    uint64_t n = L->n, pb = L->plane_bytes;
    if (k == 0) {
        for (uint64_t i = 0; i < n; ++i) {
            if (L->dtype == ORC_F32)
                ((float*)out)[i] = 0.0f;
            else
                ((double*)out)[i] = 0.0;
        }
        return ORC_OK;
    }
    uint8_t* rows = (uint8_t*)calloc((size_t)(pb * (L->B + 1) + 1), 1);
    int st = decode_unit(L, 0, rows, pb);
    for (uint32_t p0 = 0; st == ORC_OK && p0 < k; p0 += L->m) {
        uint32_t p1 = p0 + L->m < L->B ? p0 + L->m : L->B;
        st = decode_unit(L, 1 + (int)p0, rows + (uint64_t)(1 + p0) * pb, (uint64_t)(p1 - p0) * pb);
    }
    if (st != ORC_OK) {
        free(rows);
        return st;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t mag = 0;
        for (uint32_t p = 0; p < k; ++p) {
            uint64_t bit = (rows[(uint64_t)(1 + p) * pb + (uint64_t)i / 8] >> (i % 8)) & 1u;
            mag |= bit << (L->B - 1 - p);
        }
        int s = (rows[(uint64_t)i / 8] >> (i % 8)) & 1u;
        double v = ldexp((double)mag, L->e - (int)L->B);
        if (s) v = -v;
        if (L->dtype == ORC_F32)
            ((float*)out)[i] = (float)v;
        else
            ((double*)out)[i] = v;
    }
    free(rows);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* planner: tolerance -> planes per level (greedy)                            */
/* ------------------------------------------------------------------------ */
/*
 * The paper retrieves "just enough" precision segments for a requested error
 * and defers the choice to MDR.  Reading:
 *   bound(k) = sum over levels of E_l[k_l]   (summed in level order, double);
 *   from the planes already held, while bound > tol and some level is not
 *   complete, fetch one more group in the level with the largest gain
 *     (E_l[k_l] - E_l[next_l]) / bytes(next group, + sign unit if k_l = 0),
 *   ties to the smallest level; if every gain is zero, the level with the
 *   largest E_l[k_l].
 * Pins: brute force over k for one level; enumeration of all k-vectors on tiny
 * cases confirms the result meets the bound.
 */
static double plan_bound(uint32_t nlevels, uint32_t B, const double* E, const uint32_t* k)
{
    double s = 0.0;
    for (uint32_t l = 0; l < nlevels; ++l) s += E[(uint64_t)l * (B + 1) + k[l]];
    return s;
}

int orc_plan_one_step(uint32_t nlevels, uint32_t B, uint32_t m, const double* E,
                      const uint64_t* unit_bytes, uint32_t* k)
{
    int best = -1;
    double best_gain = 0.0;
    for (uint32_t l = 0; l < nlevels; ++l) {
        if (k[l] >= B) continue;
        uint32_t nxt = k[l] + m < B ? k[l] + m : B;
        const double* El = E + (uint64_t)l * (B + 1);
        const uint64_t* ub = unit_bytes + (uint64_t)l * (1 + B);
        uint64_t cost = ub[1 + k[l]] + (k[l] == 0 ? ub[0] : 0);
        if (cost == 0) cost = 1;
        double gain = (El[k[l]] - El[nxt]) / (double)cost;
        if (best < 0 || gain > best_gain) {
            best = (int)l;
            best_gain = gain;
        }
    }
    if (best < 0) return 0; /* every level complete */
    if (best_gain == 0.0) {
        best = -1;
        double worst = 0.0;
        for (uint32_t l = 0; l < nlevels; ++l) {
            if (k[l] >= B) continue;
            double el = E[(uint64_t)l * (B + 1) + k[l]];
            if (best < 0 || el > worst) {
                best = (int)l;
                worst = el;
            }
        }
    }
    k[best] = k[best] + m < B ? k[best] + m : B;
    return 1;
}

int orc_plan(uint32_t nlevels, uint32_t B, uint32_t m, const double* E,
             const uint64_t* unit_bytes, double tol, const uint32_t* k_in, uint32_t* k_out,
             double* bound)
{
    if (m < 1) return ORC_EINVAL;
    for (uint32_t l = 0; l < nlevels; ++l) k_out[l] = k_in[l];
    double b = plan_bound(nlevels, B, E, k_out);
    while (b > tol) {
        if (!orc_plan_one_step(nlevels, B, m, E, unit_bytes, k_out)) break;
        b = plan_bound(nlevels, B, E, k_out);
    }
    *bound = b;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.2: V_total = vx^2 + vy^2 + vz^2 error estimate                      */
/* ------------------------------------------------------------------------ */
/*
 * With |v - vhat| <= eps per component, |v^2 - vhat^2| = |v - vhat| |v + vhat|
 * <= eps * (2|vhat| + eps).  The estimate is the pointwise supremum of the sum
 * over the three components, evaluated in double in the order x, y, z as
 * t = eps * ((2*|vhat|) + eps), and inflated by (1 + 2^-40) to cover the
 * rounding of these few operations.
 * Pins: the paper's invariant real error <= estimate (<= tolerance), with the
 * real error computed from the originals.
 */
double orc_qoi_vtotal_tau(uint64_t n, const double* vx, const double* vy, const double* vz,
                          const double eps[3])
{
    double worst = 0.0;
    const double* v[3] = {vx, vy, vz};
    for (uint64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) {
            double a = fabs(v[c][i]);
            double t = eps[c] * ((2.0 * a) + eps[c]);
            s = s + t;
        }
        if (s > worst) worst = s;
    }
    return worst * (1.0 + ldexp(1.0, -40));
}

/*
 * The point the CP estimator (Sec. 5.2) works on: the first index (in the
 * level-concatenated order) whose sum, evaluated exactly as above, is the
 * largest.  Returns n for n = 0.
 */
uint64_t orc_qoi_vtotal_argmax(uint64_t n, const double* vx, const double* vy, const double* vz,
                               const double eps[3])
{
    double worst = -1.0;
    uint64_t at = n;
    const double* v[3] = {vx, vy, vz};
    for (uint64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) {
            double a = fabs(v[c][i]);
            double t = eps[c] * ((2.0 * a) + eps[c]);
            s = s + t;
        }
        if (s > worst) {
            worst = s;
            at = i;
        }
    }
    return at;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.2: further QoI families (error estimation for derived quantities)    */
/* ------------------------------------------------------------------------ */
/*
 * Per point, with the reconstruction's values vhat_c and L-inf bounds eps_c of
 * the variables (|v_c - vhat_c| <= eps_c), each family's raw score r(p):
 *
 *   ORC_QOI_SUMSQ      S = sum_c v_c^2 over nvars = 1..3 variables:
 *                      |S - Shat| <= D(p) = sum_c eps_c (2|vhat_c| + eps_c)
 *                      (the V_total bound; with three variables it is V_total),
 *                      r(p) = D(p).
 *   ORC_QOI_MAGNITUDE  M = sqrt(S): |M - Mhat| = |S - Shat| / (M + Mhat) <= D / Mhat
 *                      (M >= 0), and |M - Mhat| <= ||v - vhat||_2 <= sqrt(A),
 *                      A = sum_c eps_c^2 (reverse triangle inequality).  So
 *                      |M - Mhat| <= sqrt(min(A, D^2 / Shat)); the score is
 *                      r(p) = D(p)^2 / Shat(p) (+inf when Shat = 0), and the
 *                      estimate is sqrt(min(A, max_p r(p))).
 *   ORC_QOI_PRODUCT    P = v_0 v_1 (nvars = 2): P - Phat = vhat_0 e_1 +
 *                      vhat_1 e_0 + e_0 e_1 with |e_c| <= eps_c, so
 *                      |P - Phat| <= r(p) = (|vhat_0| eps_1 + |vhat_1| eps_0) + eps_0 eps_1.
 *
 * Each is evaluated in double in the order written (Shat = (vx^2 + vy^2) + vz^2),
 * and the estimate tau' (max_p r(p), or the magnitude's square root of the
 * minimum) is inflated by (1 + 2^-40) to cover the rounding of these few
 * operations.  Pins: the paper's invariant real error <= estimate <= tolerance
 * (real computed from the originals), hand-derived points, and sampled
 * perturbations inside the bounds.
 */
static double qoi_score(int kind, uint32_t nvars, const double* const* v, uint64_t i, const double eps[3])
{
    if (kind == ORC_QOI_PRODUCT) {
        double a0 = fabs(v[0][i]), a1 = fabs(v[1][i]);
        double r = (a0 * eps[1]) + (a1 * eps[0]);
        return r + (eps[0] * eps[1]);
    }
    double d = 0.0;
    for (uint32_t c = 0; c < nvars; ++c) {
        double a = fabs(v[c][i]);
        double t = eps[c] * ((2.0 * a) + eps[c]);
        d = d + t;
    }
    if (kind == ORC_QOI_SUMSQ) return d;
    double sh = 0.0;
    for (uint32_t c = 0; c < nvars; ++c) sh = sh + (v[c][i] * v[c][i]);
    if (sh == 0.0) return INFINITY;
    return (d * d) / sh;
}

/* max_p r(p) (0 for n = 0); argmax: the first point attaining it (n for n = 0) */
double orc_qoi_score_max(int kind, uint32_t nvars, uint64_t n, const double* v0, const double* v1,
                         const double* v2, const double eps[3], uint64_t* argmax)
{
    const double* v[3] = {v0, v1, v2};
    double worst = -1.0;
    uint64_t at = n;
    for (uint64_t i = 0; i < n; ++i) {
        double r = qoi_score(kind, nvars, v, i, eps);
        if (r > worst) {
            worst = r;
            at = i;
        }
    }
    if (argmax) *argmax = at;
    return n ? worst : 0.0;
}

/* the estimate tau' from the largest score */
double orc_qoi_estimate(int kind, uint32_t nvars, double score_max, const double eps[3])
{
    double t = score_max;
    if (kind == ORC_QOI_MAGNITUDE) {
        double a = 0.0;
        for (uint32_t c = 0; c < nvars; ++c) a = a + (eps[c] * eps[c]);
        t = sqrt(score_max < a ? score_max : a);
    }
    return t * (1.0 + ldexp(1.0, -40));
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.1 serialization (container format of this project)                 */
/* ------------------------------------------------------------------------ */
/*
 * Little-endian throughout.
 * Variable header (56 bytes):
 *   0 u32 magic 0x3152444D ("MDR1")  4 u8 version=1  5 u8 dtype  6 u8 B  7 u8 m
 *   8 u32 nlevels  12 u32 t_cr_milli  16 u64 t_s  24 u32 huf_chunk  28 u32 huf_lmax
 *   32 i32 force_method  36 u32 0  40 u64 total blob bytes  48 u32 crc32(bytes 0..47)
 *   52 u32 0
 * Per level:
 *   u64 n | i32 e | u32 nstreams=1+B | f64 vmin | f64 vmax | f64 vmaxabs | f64 E[B+1]
 *   nstreams x { u8 method | u8 0,0,0 | u32 crc32(payload) | u64 bytes }
 *   u32 crc32(record so far) | u32 0
 *   payloads in table order, each zero padded to a multiple of 8 bytes.
 */
static uint64_t pad8(uint64_t v)
{
    return (v + 7) & ~(uint64_t)7;
}

int orc_serialize(orc_level* const* levels, uint32_t nlevels, const orc_params* prm, uint8_t* out,
                  uint64_t cap, uint64_t* used)
{
    if (nlevels == 0) return ORC_EINVAL;
    uint32_t B = levels[0]->B;
    uint64_t total = 56;
    for (uint32_t l = 0; l < nlevels; ++l) {
        const orc_level* L = levels[l];
        if (L->B != B || L->dtype != levels[0]->dtype) return ORC_EINVAL;
        total += 16 + 24 + 8 * (uint64_t)(B + 1) + 16 * (uint64_t)(1 + B) + 8;
        for (uint32_t s = 0; s < 1 + B; ++s)
            if (L->method[s] != ORC_PLACEHOLDER) total += pad8(L->bytes[s]);
    }
    *used = total;
    if (out == NULL || cap < total) return cap == 0 ? ORC_OK : ORC_ENOMEM;
    memset(out, 0, (size_t)total);
    put_u32(out + 0, 0x3152444Du);
    out[4] = 1;
    out[5] = (uint8_t)levels[0]->dtype;
    out[6] = (uint8_t)B;
    out[7] = (uint8_t)levels[0]->m;
    put_u32(out + 8, nlevels);
    put_u32(out + 12, prm->t_cr_milli);
    put_u64(out + 16, prm->t_s);
    put_u32(out + 24, prm->huf_chunk);
    put_u32(out + 28, prm->huf_lmax);
    put_u32(out + 32, (uint32_t)prm->force_method);
    put_u64(out + 40, total);
    put_u32(out + 48, orc_crc32(out, 48));
    uint64_t pos = 56;
    for (uint32_t l = 0; l < nlevels; ++l) {
        const orc_level* L = levels[l];
        uint64_t rec = pos;
        put_u64(out + pos, L->n);
        put_u32(out + pos + 8, (uint32_t)L->e);
        put_u32(out + pos + 12, 1 + B);
        pos += 16;
        double meta[3] = {L->vmin, L->vmax, L->vmaxabs};
        for (int i = 0; i < 3; ++i) {
            uint64_t bits;
            memcpy(&bits, &meta[i], 8);
            put_u64(out + pos, bits);
            pos += 8;
        }
        for (uint32_t k = 0; k <= B; ++k) {
            uint64_t bits;
            memcpy(&bits, &L->E[k], 8);
            put_u64(out + pos, bits);
            pos += 8;
        }
        for (uint32_t s = 0; s < 1 + B; ++s) {
            int meth = L->method[s];
            uint64_t nb = meth == ORC_PLACEHOLDER ? 0 : L->bytes[s];
            out[pos] = (uint8_t)meth;
            put_u32(out + pos + 4, nb ? orc_crc32(L->data[s], nb) : orc_crc32(NULL, 0));
            put_u64(out + pos + 8, nb);
            pos += 16;
        }
        put_u32(out + pos, orc_crc32(out + rec, pos - rec));
        pos += 8;
        for (uint32_t s = 0; s < 1 + B; ++s) {
            if (L->method[s] == ORC_PLACEHOLDER) continue;
            memcpy(out + pos, L->data[s], (size_t)L->bytes[s]);
            pos += pad8(L->bytes[s]);
        }
    }
    return pos == total ? ORC_OK : ORC_EINVAL;
}
