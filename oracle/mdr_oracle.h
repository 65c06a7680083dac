/*
 * mdr_oracle.h -- plain CPU oracle for the bitplane refactor / retrieve path
 * of HP-MDR (arXiv 2505.00227).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library.  The product
 * library (paper_2505_00227_amd) shares no code, header or table with it.
 *
 * Every function is the plain, slow definition of one step of the method:
 *   - exponent alignment and fixed-point sign/magnitude     (Sec. 3, Alg. 1 step 1)
 *   - bitplane extraction, most significant plane first     (Sec. 3, Alg. 1 loop)
 *   - exact per-plane L-infinity error table                (not in the paper; the
 *     progressive-retrieval error estimate of MDR it builds on, Sec. 2.2)
 *   - Huffman / RLE / direct copy and the hybrid selection  (Sec. 4, Alg. 2)
 *   - tolerance -> planes greedy planner                    (Sec. 1/5, retrieval to a bound)
 *   - V_total QoI bound and the MAPE loop                   (Sec. 5.2, Alg. 3)
 *   - the serialized container                              (Sec. 5.1, serialization)
 *
 * Parity status of each function is stated at its definition in mdr_oracle.c.
 */
#ifndef MDR_ORACLE_H
#define MDR_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F64 = 1 };
enum { ORC_DC = 0, ORC_RLE = 1, ORC_HUF = 2, ORC_PLACEHOLDER = 3 };
enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EUNSUP = 2, ORC_ENOMEM = 3, ORC_ECORRUPT = 5 };

typedef struct {
    uint32_t group_planes;  /* m: planes merged per lossless group (Alg. 2)        */
    uint32_t t_cr_milli;    /* T_cr x 1000                                          */
    uint64_t t_s;           /* T_s in bytes                                         */
    uint32_t huf_chunk;     /* byte symbols per independently decodable chunk       */
    uint32_t huf_lmax;      /* longest Huffman code allowed                         */
    int32_t force_method;   /* -1: Alg. 2 decides; else every unit uses this method */
} orc_params;

typedef struct orc_level orc_level; /* one refactored level (opaque) */

void orc_set_threads(int nthreads);
int orc_get_threads(void);

/* ---- step functions (each usable on its own by the tests) ---- */
int orc_stats(const void* x, uint64_t n, int dtype, int32_t* e, double* vmin, double* vmax,
              double* vmaxabs);
void orc_fixed_point(const void* x, uint64_t n, int dtype, int32_t e, uint32_t B, uint64_t* mag,
                     uint8_t* sign);
uint64_t orc_plane_bytes(uint64_t n, uint32_t W);
void orc_bitplanes(const uint64_t* mag, const uint8_t* sign, uint64_t n, uint32_t B, uint32_t W,
                   uint8_t* rows /* (B+1) * plane_bytes; row 0 = sign */);
void orc_error_table(const void* x, const uint64_t* mag, uint64_t n, int dtype, int32_t e,
                     uint32_t B, double* E /* B+1 */);

int orc_huffman_lengths(const uint64_t* freq /* 256 */, uint32_t lmax, uint8_t* len /* 256 */);
void orc_huffman_codes(const uint8_t* len, uint32_t* code /* 256 */);
uint64_t orc_huffman_estimate(const uint64_t* freq, const uint8_t* len, uint64_t S, uint32_t chunk);
uint64_t orc_huffman_encoded_size(const uint8_t* g, uint64_t S, uint32_t chunk, uint32_t lmax);
int orc_huffman_encode(const uint8_t* g, uint64_t S, uint32_t chunk, uint32_t lmax, uint8_t* out,
                       uint64_t cap, uint64_t* used);
int orc_huffman_decode(const uint8_t* p, uint64_t bytes, uint32_t chunk, uint8_t* g, uint64_t S);

uint64_t orc_rle_runs(const uint8_t* g, uint64_t S, uint32_t wbytes);
uint64_t orc_rle_estimate(uint64_t nruns, uint32_t wbytes);
int orc_rle_encode(const uint8_t* g, uint64_t S, uint32_t wbytes, uint8_t* out, uint64_t cap,
                   uint64_t* used);
int orc_rle_decode(const uint8_t* p, uint64_t bytes, uint32_t wbytes, uint8_t* g, uint64_t S);

int orc_select(uint64_t S, uint64_t est_huf, uint64_t est_rle, const orc_params* prm);

uint32_t orc_crc32(const uint8_t* p, uint64_t n);

/* ---- one level: refactor, inspect, reconstruct ---- */
int orc_refactor_level(const void* x, uint64_t n, int dtype, uint32_t B, const orc_params* prm,
                       orc_level** out);
void orc_level_free(orc_level* L);
int orc_level_info(const orc_level* L, uint64_t* n, int32_t* e, double* vmin, double* vmax,
                   double* vmaxabs, double* E /* B+1 */);
int orc_level_stream(const orc_level* L, int32_t stream /* -1 sign, 0..B-1 planes */,
                     int32_t* method, uint64_t* bytes, const uint8_t** data, uint64_t* est_huf,
                     uint64_t* est_rle);
const uint8_t* orc_level_rows(const orc_level* L, uint64_t* plane_bytes);
int orc_reconstruct(const orc_level* L, uint32_t k, void* out);

/* ---- planner and QoI (whole variable = list of levels) ---- */
int orc_plan(uint32_t nlevels, uint32_t B, uint32_t m, const double* E /* nlevels*(B+1) */,
             const uint64_t* unit_bytes /* nlevels*(1+B): sign, then per plane (0 if placeholder) */,
             double tol, const uint32_t* k_in, uint32_t* k_out, double* bound);
int orc_plan_one_step(uint32_t nlevels, uint32_t B, uint32_t m, const double* E,
                      const uint64_t* unit_bytes, uint32_t* k /* in/out */);
void orc_abl_planes(int interleaved, const uint32_t* in, uint64_t n, uint32_t* planes, uint64_t words);
/* QoI families of Sec. 5.2 beyond V_total (see the definitions in mdr_oracle.c) */
enum { ORC_QOI_SUMSQ = 0, ORC_QOI_MAGNITUDE = 1, ORC_QOI_PRODUCT = 2 };
double orc_qoi_score_max(int kind, uint32_t nvars, uint64_t n, const double* v0, const double* v1,
                         const double* v2, const double eps[3], uint64_t* argmax);
double orc_qoi_estimate(int kind, uint32_t nvars, double score_max, const double eps[3]);
uint64_t orc_qoi_vtotal_argmax(uint64_t n, const double* vx, const double* vy, const double* vz,
                               const double eps[3]);
double orc_qoi_vtotal_tau(uint64_t n, const double* vx, const double* vy, const double* vz,
                          const double eps[3]);

/* ---- serialization ---- */
int orc_serialize(orc_level* const* levels, uint32_t nlevels, const orc_params* prm, uint8_t* out,
                  uint64_t cap, uint64_t* used);

#ifdef __cplusplus
}
#endif
#endif
