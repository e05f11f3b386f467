/*
 * CPU oracle for the error-bounded Lorenzo + Huffman compression path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP implementation: every step is written out here
 * again, slowly and plainly, in the order the method defines it.
 *
 * What it computes (FZModules: Sec. 3.1 the cuSZ design, Sec. 3.2 the module
 * interfaces, Sec. 3.3 the FZMod-Default pipeline, Sec. 4.2 the metrics):
 *   1. error-bound resolution: absolute, or value-range relative
 *      (Sec. 3.2: the relative mode needs the data minimum and maximum);
 *   2. prequantisation of every value onto the grid of step 2*eb
 *      (dual quantisation of cuSZ, Sec. 3.1);
 *   3. block-local first-order Lorenzo prediction on the integer grid,
 *      residual = backward difference along every axis (Sec. 3.1, 3.2);
 *   4. post-quantisation: residuals inside the radius become integer codes,
 *      the rest are stored as outliers (Sec. 3.1: unpredictable values are
 *      kept as outliers; Sec. 3.3.1 outlier handling);
 *   5. a histogram of the codes (Sec. 3.2: the Huffman encoder needs it);
 *   6. a length-limited minimum-redundancy (Huffman) code built from the
 *      histogram, in canonical form (Sec. 3.2: Huffman for the best ratio);
 *   7. chunked Huffman encoding, one chunk per block (Sec. 3.3);
 *   8. the container; decoding, outlier scatter and inverse Lorenzo
 *      (prefix sums) with dequantisation (Sec. 1 and Sec. 3.3.1 describe
 *      decompression as Huffman decoding plus outlier scatter).
 * The paper leaves every bit-level choice to the cuSZ papers; the readings
 * taken here (block shapes, code layout, tie rules, container layout, the
 * lossless patches that make the bound strict) are the ones the HIP path
 * must reproduce and are listed with the design notes of the project.
 *
 * Pins: tests/test_oracle_*.py check this file against brute force on tiny
 * inputs, closed forms, textbook Huffman costs, invariants (max error <= eb,
 * histogram sums to N, Kraft equality, round trip) and hand-made examples.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math (no contraction,
 * no fast math, SSE2 doubles, round-to-nearest-even).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------- errors */
#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_EB (-2)
#define ORC_ERR_NONFINITE (-3)
#define ORC_ERR_CAPACITY (-4)
#define ORC_ERR_CORRUPT (-5)
#define ORC_ERR_NOMEM (-7)
#define ORC_ERR_UNSUPPORTED (-8)

/* --------------------------------------------------------------- constants */
#define ORC_RADIUS 512        /* codes 1..1023 hold residuals -511..511      */
#define ORC_NBINS 1024        /* code 0 marks an outlier                     */
#define ORC_LMAX 12           /* longest codeword                            */
#define ORC_HDR 128           /* container header bytes                      */
#define ORC_BLOCK_ELEMS 512   /* every block holds at most 512 values        */
#define ORC_MAGIC 0x314D5A46u /* bytes 'F' 'Z' 'M' '1'                       */
#define ORC_VERSION 1
#define ORC_FLAG_SHUFFLE 2    /* header flag: bit-shuffle codec container    */

/* ------------------------------------------------------------ block shapes
 * 1D blocks are 512 long, 2D blocks 32 (x) by 16 (y), 3D blocks 8x8x8.
 * dims[0] is the fastest-varying axis.  Edge blocks are truncated.        */
static void block_shape(int ndim, int bs[3]) {
    if (ndim == 1) { bs[0] = 512; bs[1] = 1; bs[2] = 1; }
    else if (ndim == 2) { bs[0] = 32; bs[1] = 16; bs[2] = 1; }
    else { bs[0] = 8; bs[1] = 8; bs[2] = 8; }
}

typedef struct {
    int ndim;
    uint64_t n[3];   /* field extent per axis (unused axes are 1) */
    int bs[3];       /* block extent per axis                     */
    uint64_t nb[3];  /* number of blocks per axis                 */
    uint64_t nblocks;
    uint64_t N;
} geom_t;

static int make_geom(int ndim, const uint64_t dims[3], geom_t *g) {
    if (ndim < 1 || ndim > 3) return ORC_ERR_ARG;
    g->ndim = ndim;
    for (int a = 0; a < 3; a++) g->n[a] = (a < ndim) ? dims[a] : 1;
    for (int a = 0; a < 3; a++) if (g->n[a] < 1) return ORC_ERR_ARG;
    block_shape(ndim, g->bs);
    g->N = g->n[0] * g->n[1] * g->n[2];
    if (g->n[0] > 0xFFFFFFFFull || g->n[1] > 0xFFFFFFFFull || g->n[2] > 0xFFFFFFFFull) return ORC_ERR_ARG;
    for (int a = 0; a < 3; a++) g->nb[a] = (g->n[a] + g->bs[a] - 1) / g->bs[a];
    g->nblocks = g->nb[0] * g->nb[1] * g->nb[2];
    /* positions are u32: block index * 512 + in-block offset */
    if (g->nblocks > (1ull << 23)) return ORC_ERR_ARG;
    return ORC_OK;
}

/* row-major index of (x, y, z) */
static uint64_t rm(const geom_t *g, uint64_t x, uint64_t y, uint64_t z) {
    return x + g->n[0] * (y + g->n[1] * z);
}

/* --------------------------------------------- step 1: error-bound resolution
 * Absolute mode: eb_abs = eb.  Relative mode: eb_abs = eb * (max - min),
 * range taken in double; a constant field (range 0) uses eb itself.
 * (Sec. 3.2 preprocessors; Sec. 4.2 value-range relative bound.)         */
int orc_eb_abs(const float *x, uint64_t N, int mode, double eb, double *eb_abs) {
    if (!(eb > 0.0) || !isfinite(eb)) return ORC_ERR_EB;
    for (uint64_t i = 0; i < N; i++)
        if (!isfinite(x[i])) return ORC_ERR_NONFINITE;
    double e;
    if (mode == 0) {
        e = eb;
    } else if (mode == 1) {
        float lo = x[0], hi = x[0];
        for (uint64_t i = 1; i < N; i++) {
            if (x[i] < lo) lo = x[i];
            if (x[i] > hi) hi = x[i];
        }
        double range = (double)hi - (double)lo;
        e = (range > 0.0) ? eb * range : eb;
    } else {
        return ORC_ERR_ARG;
    }
    if (!(e >= 1e-300 && e <= 1e300)) return ORC_ERR_EB;
    *eb_abs = e;
    return ORC_OK;
}

/* -------------------------------------------------- step 2: prequantisation
 * q = round-half-even(x / (2 eb_abs)) computed as x * (1 / (2 eb_abs)) in
 * double.  A value is a lossless patch when the grid value is out of the
 * 2^24 range (q is then 0) or when the reconstruction rounded to float
 * misses the bound (q is kept).  The bound is inclusive.                  */
void orc_prequant(const float *x, uint64_t N, double eb_abs, int32_t *q, uint8_t *patch) {
    double e2 = 2.0 * eb_abs;
    double inv = 1.0 / e2;
    for (uint64_t i = 0; i < N; i++) {
        double t = (double)x[i] * inv;
        if (fabs(t) >= 16777216.0) {
            q[i] = 0;
            patch[i] = 1;
        } else {
            int32_t qi = (int32_t)nearbyint(t);
            float xh = (float)((double)qi * e2);
            q[i] = qi;
            patch[i] = fabs((double)x[i] - (double)xh) > eb_abs ? 1 : 0;
        }
    }
}

/* dequantisation of one grid value */
static float dequant(int32_t qv, double e2) { return (float)((double)qv * e2); }

/* ------------------------------------- step 3: block-local Lorenzo residual
 * Neighbours outside the element's own block count as zero.
 * 1D: d = q - q[x-1]
 * 2D: d = q - q[x-1] - q[y-1] + q[x-1,y-1]
 * 3D: d = q - q[x-1] - q[y-1] - q[z-1] + q[x-1,y-1] + q[x-1,z-1]
 *         + q[y-1,z-1] - q[x-1,y-1,z-1]
 * Output is in row-major order like the input.                           */
static int32_t qnb(const geom_t *g, const int32_t *q, uint64_t x, uint64_t y, uint64_t z,
                   int dx, int dy, int dz) {
    /* q at (x-dx, y-dy, z-dz) if that point lies in the same block, else 0 */
    uint64_t lx = x % (uint64_t)g->bs[0], ly = y % (uint64_t)g->bs[1], lz = z % (uint64_t)g->bs[2];
    if ((uint64_t)dx > lx || (uint64_t)dy > ly || (uint64_t)dz > lz) return 0;
    return q[rm(g, x - dx, y - dy, z - dz)];
}

void orc_lorenzo1(const int32_t *q, int ndim, const uint64_t dims[3], int32_t *delta) {
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return;
    for (uint64_t z = 0; z < g.n[2]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[0]; x++) {
                int32_t d;
                if (ndim == 1) {
                    d = qnb(&g, q, x, y, z, 0, 0, 0) - qnb(&g, q, x, y, z, 1, 0, 0);
                } else if (ndim == 2) {
                    d = qnb(&g, q, x, y, z, 0, 0, 0) - qnb(&g, q, x, y, z, 1, 0, 0)
                      - qnb(&g, q, x, y, z, 0, 1, 0) + qnb(&g, q, x, y, z, 1, 1, 0);
                } else {
                    d = qnb(&g, q, x, y, z, 0, 0, 0) - qnb(&g, q, x, y, z, 1, 0, 0)
                      - qnb(&g, q, x, y, z, 0, 1, 0) - qnb(&g, q, x, y, z, 0, 0, 1)
                      + qnb(&g, q, x, y, z, 1, 1, 0) + qnb(&g, q, x, y, z, 1, 0, 1)
                      + qnb(&g, q, x, y, z, 0, 1, 1) - qnb(&g, q, x, y, z, 1, 1, 1);
                }
                delta[rm(&g, x, y, z)] = d;
            }
}

/* Inverse: inclusive prefix sums inside each block, along x, then y, then z. */
void orc_lorenzo1_inverse(const int32_t *delta, int ndim, const uint64_t dims[3], int32_t *q) {
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return;
    memcpy(q, delta, sizeof(int32_t) * g.N);
    for (uint64_t z = 0; z < g.n[2]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[0]; x++)
                if (x % g.bs[0] != 0) q[rm(&g, x, y, z)] += q[rm(&g, x - 1, y, z)];
    for (uint64_t z = 0; z < g.n[2]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[0]; x++)
                if (y % g.bs[1] != 0) q[rm(&g, x, y, z)] += q[rm(&g, x, y - 1, z)];
    for (uint64_t z = 0; z < g.n[2]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[0]; x++)
                if (z % g.bs[2] != 0) q[rm(&g, x, y, z)] += q[rm(&g, x, y, z - 1)];
}

/* --------------------------------------------------- block-major traversal
 * Blocks in row-major order over the block grid (block x fastest); inside a
 * block, elements x fastest, then y, then z, over the block's real extent.
 * An element's position is  block_index * 512 + lx + bs0 * (ly + bs1 * lz)
 * (full-block strides, so truncated blocks leave gaps in the numbering).   */
typedef struct {
    uint64_t idx;  /* row-major index */
    uint32_t pos;  /* position        */
} elem_ref;

/* Fill refs[] with every element in block-major order; returns count (= N). */
static uint64_t block_major_order(const geom_t *g, elem_ref *refs, uint32_t *block_count) {
    uint64_t k = 0, b = 0;
    for (uint64_t bz = 0; bz < g->nb[2]; bz++)
        for (uint64_t by = 0; by < g->nb[1]; by++)
            for (uint64_t bx = 0; bx < g->nb[0]; bx++, b++) {
                uint32_t cnt = 0;
                for (int lz = 0; lz < g->bs[2]; lz++)
                    for (int ly = 0; ly < g->bs[1]; ly++)
                        for (int lx = 0; lx < g->bs[0]; lx++) {
                            uint64_t x = bx * g->bs[0] + lx, y = by * g->bs[1] + ly, z = bz * g->bs[2] + lz;
                            if (x >= g->n[0] || y >= g->n[1] || z >= g->n[2]) continue;
                            refs[k].idx = rm(g, x, y, z);
                            refs[k].pos = (uint32_t)(b * ORC_BLOCK_ELEMS + lx + g->bs[0] * (ly + g->bs[1] * lz));
                            k++;
                            cnt++;
                        }
                block_count[b] = cnt;
            }
    return k;
}

/* ---------------------------------------------- step 4: post-quantisation
 * |d| < radius -> code d + radius (1..1023); otherwise code 0 and outlier. */
static uint16_t postquant(int32_t d) {
    if (d > -ORC_RADIUS && d < ORC_RADIUS) return (uint16_t)(d + ORC_RADIUS);
    return 0;
}

/* ------------------------------------------------------- step 5: histogram */
void orc_histogram(const uint16_t *codes, uint64_t n, uint32_t *hist) {
    memset(hist, 0, sizeof(uint32_t) * ORC_NBINS);
    for (uint64_t i = 0; i < n; i++) hist[codes[i]]++;
}

/* ---------------------------------- step 6: length-limited Huffman lengths
 * Minimum-redundancy prefix code with every length <= lmax, by the
 * package-merge method (Larmore & Hirschberg, 1990), written out plainly:
 *
 *   leaves   : used symbols sorted by (count, symbol) ascending;
 *   list[lmax] = leaves;
 *   list[l]  = merge of leaves and packages of list[l+1], where package j
 *              is item 2j + item 2j+1 of list[l+1] (an unpaired last item is
 *              dropped); equal weights put the leaf first, packages keep
 *              their order;
 *   select the first 2n-2 items of list[1]; the selected packages of
 *   list[l] stand for the first 2*(#packages) items of list[l+1];
 *   a symbol's length is the number of levels at which it was selected.
 *
 * A single used symbol gets a companion of weight 0 (the smallest unused
 * symbol) so that both get length 1 and the Kraft sum is exactly 1.
 * Returns 0, or -1 if lmax cannot hold the alphabet.                      */
typedef struct {
    uint64_t w;
    int leaf;   /* leaf rank in the sorted leaf list, or -1 for a package */
} pm_item;

int orc_codebook_lmax(const uint32_t *hist, int nsym, int lmax, uint8_t *len) {
    int *sym = (int *)malloc(sizeof(int) * (nsym + 1));
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (nsym + 1));
    int n = 0;
    for (int s = 0; s < nsym; s++) len[s] = 0;
    for (int s = 0; s < nsym; s++)
        if (hist[s] > 0) { sym[n] = s; w[n] = hist[s]; n++; }
    if (n == 0) { free(sym); free(w); return 0; }
    if (n == 1) {
        int ph = 0;
        while (ph < nsym && hist[ph] > 0) ph++;
        if (ph == nsym) { len[sym[0]] = 1; free(sym); free(w); return 0; }
        len[sym[0]] = 1;
        len[ph] = 1;
        free(sym); free(w);
        return 0;
    }
    if ((1ull << lmax) < (uint64_t)n) { free(sym); free(w); return -1; }
    /* sort leaves by (weight, symbol): insertion sort keeps it plain */
    for (int i = 1; i < n; i++) {
        int s = sym[i];
        uint64_t ws = w[i];
        int j = i - 1;
        while (j >= 0 && (w[j] > ws || (w[j] == ws && sym[j] > s))) {
            sym[j + 1] = sym[j];
            w[j + 1] = w[j];
            j--;
        }
        sym[j + 1] = s;
        w[j + 1] = ws;
    }
    /* lists[l] for l = 1..lmax */
    int maxlen = 2 * n;
    pm_item **lists = (pm_item **)calloc(lmax + 1, sizeof(pm_item *));
    int *llen = (int *)calloc(lmax + 1, sizeof(int));
    for (int l = 1; l <= lmax; l++) lists[l] = (pm_item *)malloc(sizeof(pm_item) * maxlen);
    for (int i = 0; i < n; i++) { lists[lmax][i].w = w[i]; lists[lmax][i].leaf = i; }
    llen[lmax] = n;
    for (int l = lmax - 1; l >= 1; l--) {
        const pm_item *prev = lists[l + 1];
        int np = llen[l + 1] / 2;
        int a = 0, p = 0, k = 0;
        while (a < n || p < np) {
            uint64_t pw = (p < np) ? prev[2 * p].w + prev[2 * p + 1].w : 0;
            if (p >= np || (a < n && w[a] <= pw)) {
                lists[l][k].w = w[a];
                lists[l][k].leaf = a;
                a++;
            } else {
                lists[l][k].w = pw;
                lists[l][k].leaf = -1;
                p++;
            }
            k++;
        }
        llen[l] = k;
    }
    /* selection, top level down */
    int take = 2 * n - 2;
    for (int l = 1; l <= lmax && take > 0; l++) {
        int packages = 0;
        for (int i = 0; i < take; i++) {
            if (lists[l][i].leaf >= 0) len[sym[lists[l][i].leaf]]++;
            else packages++;
        }
        take = 2 * packages;
    }
    for (int l = 1; l <= lmax; l++) free(lists[l]);
    free(lists); free(llen); free(sym); free(w);
    return 0;
}

int orc_codebook(const uint32_t *hist, uint8_t *len) {
    return orc_codebook_lmax(hist, ORC_NBINS, ORC_LMAX, len);
}

/* Canonical codewords: used symbols ordered by (length, symbol); the first
 * gets 0, each next one (previous + 1) shifted left by the length step.   */
void orc_canonical(const uint8_t *len, int nsym, uint32_t *code) {
    uint32_t c = 0;
    int prev_len = 0, first = 1;
    for (int L = 1; L <= 32; L++)
        for (int s = 0; s < nsym; s++) {
            if (len[s] != L) continue;
            if (first) { c = 0; first = 0; }
            else c = (c + 1) << (L - prev_len);
            code[s] = c;
            prev_len = L;
        }
    for (int s = 0; s < nsym; s++) if (len[s] == 0) code[s] = 0;
}

/* ------------------------------------------------------------- bit writer
 * Bits are packed MSB-first into 32-bit words (bit 31 first); words are
 * stored little-endian.                                                   */
typedef struct {
    uint32_t *words;
    uint64_t nbits;
} bitw;

static void put_bits(bitw *bw, uint32_t value, int nbits) {
    for (int i = nbits - 1; i >= 0; i--) {
        uint32_t bit = (value >> i) & 1u;
        uint64_t w = bw->nbits / 32;
        int off = 31 - (int)(bw->nbits % 32);
        if (off == 31) bw->words[w] = 0;
        bw->words[w] |= bit << off;
        bw->nbits++;
    }
}

/* --------------------------------------------------- little-endian helpers */
static void st16(uint8_t *p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void st32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void st64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint16_t ld16(const uint8_t *p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t ld32(const uint8_t *p) {
    uint32_t v = 0;
    for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i);
    return v;
}
static uint64_t ld64(const uint8_t *p) {
    uint64_t v = 0;
    for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}
static uint64_t a16(uint64_t v) { return (v + 15) & ~15ull; }
static uint64_t f64bits(double d) { uint64_t u; memcpy(&u, &d, 8); return u; }
static double bitsf64(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }

/* ------------------------------------------------ per-block predictors
 * A block is predicted by one of:
 *   P0: first-order Lorenzo, the residual above (backward difference along
 *       every axis);
 *   P1: second-order Lorenzo, the backward difference applied twice along
 *       every axis: weights (1, -2, 1) per axis, 27 neighbours in 3D;
 *   P2: a linear fit over the block in integer fixed point.
 * Neighbours outside the block are zero for P0 and P1.  (The paper names
 * Lorenzo extrapolation and linear regression as the SZ-family predictors,
 * Sec. 2.1, and leaves predictor choice to future "auto-selection",
 * Sec. 5.)                                                               */
#define ORC_P0 0
#define ORC_P1 1
#define ORC_P2 2

static void block_coords(const geom_t *g, uint64_t b, uint64_t bc[3], int ext[3]) {
    bc[0] = b % g->nb[0];
    bc[1] = (b / g->nb[0]) % g->nb[1];
    bc[2] = b / (g->nb[0] * g->nb[1]);
    for (int a = 0; a < 3; a++) {
        uint64_t o = bc[a] * (uint64_t)g->bs[a];
        uint64_t e = g->n[a] - o;
        ext[a] = (int)(e < (uint64_t)g->bs[a] ? e : (uint64_t)g->bs[a]);
    }
}

static int32_t lorenzo2_at(const geom_t *g, const int32_t *q, uint64_t x, uint64_t y, uint64_t z) {
    static const int w[3] = {1, -2, 1};
    int nz = g->ndim >= 3 ? 3 : 1, ny = g->ndim >= 2 ? 3 : 1;
    int64_t d = 0;
    for (int dz = 0; dz < nz; dz++)
        for (int dy = 0; dy < ny; dy++)
            for (int dx = 0; dx < 3; dx++) {
                int64_t c = (int64_t)w[dx] * (g->ndim >= 2 ? w[dy] : 1) * (g->ndim >= 3 ? w[dz] : 1);
                d += c * qnb(g, q, x, y, z, dx, dy, dz);
            }
    return (int32_t)d;
}

/* round half away from zero; b > 0 */
static int64_t rdiv(int64_t a, int64_t b) {
    if (a >= 0) return (a + b / 2) / b;
    return -((-a + b / 2) / b);
}

static int32_t clamp32(int64_t v) {
    if (v > INT32_MAX) return INT32_MAX;
    if (v < INT32_MIN) return INT32_MIN;
    return (int32_t)v;
}

/* Least-squares plane over the block's real values with centred
 * coordinates u = 2 lx - (ex - 1) (likewise v, w): the normal equations
 * decouple, A = S0 / n, Bx = Su / sum(u^2), ...  Stored with 8 fractional
 * bits, rounded half away from zero, clamped to int32.                   */
static void regression_coeffs(const geom_t *g, const int32_t *q, uint64_t b, int32_t coef[4]) {
    uint64_t bc[3];
    int ext[3];
    block_coords(g, b, bc, ext);
    int64_t s0 = 0, su[3] = {0, 0, 0};
    for (int lz = 0; lz < ext[2]; lz++)
        for (int ly = 0; ly < ext[1]; ly++)
            for (int lx = 0; lx < ext[0]; lx++) {
                int64_t v = q[rm(g, bc[0] * g->bs[0] + lx, bc[1] * g->bs[1] + ly, bc[2] * g->bs[2] + lz)];
                int l[3] = {lx, ly, lz};
                s0 += v;
                for (int a = 0; a < 3; a++) su[a] += (int64_t)(2 * l[a] - (ext[a] - 1)) * v;
            }
    int64_t n = (int64_t)ext[0] * ext[1] * ext[2];
    coef[0] = clamp32(rdiv(s0 * 256, n));
    for (int a = 0; a < 3; a++) {
        /* sum of u^2 over the block: ext_a (ext_a^2 - 1) / 3 per line, times the other extents */
        int64_t d = (int64_t)ext[a] * ((int64_t)ext[a] * ext[a] - 1) / 3 * (n / ext[a]);
        coef[1 + a] = d > 0 ? clamp32(rdiv(su[a] * 256, d)) : 0;
    }
}

static int32_t regression_pred(const int32_t coef[4], const int ext[3], int lx, int ly, int lz) {
    int64_t s = (int64_t)coef[0] + (int64_t)coef[1] * (2 * lx - (ext[0] - 1)) +
                (int64_t)coef[2] * (2 * ly - (ext[1] - 1)) + (int64_t)coef[3] * (2 * lz - (ext[2] - 1));
    /* floor((s + 128) / 256) */
    int64_t t = s + 128;
    return (int32_t)(t >= 0 ? t / 256 : -((-t + 255) / 256));
}

/* residual of the value at (x, y, z) under predictor p (coef: P2 only) */
/* ------------------------------------------ interpolation predictor (G-Interp)
 * The prediction of the quality-oriented pipeline (Sec. 3.2, Sec. 3.3
 * FZMod-Quality: the G-Interp spline interpolator of cuSZ-i in place of the
 * Lorenzo predictor).  The paper gives no formula; this is the reading the
 * project fixes, on the prequantised integers (dual quantisation, as the
 * Lorenzo path), over the whole field (not block-local):
 *   - anchors: points whose every coordinate is a multiple of 8, predicted
 *     by first-order Lorenzo on the grid of anchors (neighbours 8 apart,
 *     zero outside the field);
 *   - levels of stride s = 4, 2, 1: a point whose coordinates are all
 *     multiples of s, not all of 2s, is interpolated along its axis a: x if
 *     x is an odd multiple of s, else y if y is, else z (for a level the
 *     z-odd points come first, then the y-odd, then the x-odd, so every
 *     neighbour used is known before);
 *   - along a, with neighbours at a -/+ s and a -/+ 3s: cubic when both
 *     3s neighbours lie in the field, floor((-q[-3s] + 9 q[-s] + 9 q[+s]
 *     - q[+3s] + 8) / 16); else linear when a + s lies in the field,
 *     floor((q[-s] + q[+s] + 1) / 2); else q[-s];
 *   - residual = q - prediction (modulo 2^32).
 * Codes, outliers, patches and Huffman chunks (8^3 blocks, block-major
 * positions) are those of the Lorenzo path; decoding rebuilds the anchors by
 * prefix sums over the anchor grid, then the levels in the order above.   */
#define ORC_P_INTERP 5

static int64_t floordiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

/* axis interpolated at (c[0], c[1], c[2]) and its stride, or -1 for an anchor */
static int interp_axis(const geom_t *g, const uint64_t c[3], int *stride) {
    for (int s = 4; s >= 1; s >>= 1) {
        int all = 1;
        for (int a = 0; a < g->ndim; a++) if (c[a] % (uint64_t)s) all = 0;
        if (!all) continue;
        int coarse = 1;
        for (int a = 0; a < g->ndim; a++) if (c[a] % (uint64_t)(2 * s)) coarse = 0;
        if (coarse) {
            if (s == 4) { *stride = 8; return -1; }
            continue;
        }
        *stride = s;
        for (int a = 0; a < g->ndim; a++) if (c[a] % (uint64_t)(2 * s)) return a;
    }
    *stride = 8;
    return -1;
}

static int32_t qat(const geom_t *g, const int32_t *q, const uint64_t c[3]) { return q[rm(g, c[0], c[1], c[2])]; }

static int32_t interp_pred(const geom_t *g, const int32_t *q, uint64_t x, uint64_t y, uint64_t z) {
    uint64_t c[3] = {x, y, z};
    int s;
    int a = interp_axis(g, c, &s);
    if (a < 0) {
        /* anchor: first-order Lorenzo on the anchor grid */
        int64_t pred = 0;
        for (int m = 1; m < (1 << g->ndim); m++) {
            uint64_t d[3] = {c[0], c[1], c[2]};
            int ok = 1, bits = 0;
            for (int k = 0; k < g->ndim; k++)
                if (m >> k & 1) {
                    if (d[k] < 8) ok = 0; else d[k] -= 8;
                    bits++;
                }
            if (ok) pred += (bits & 1) ? qat(g, q, d) : -(int64_t)qat(g, q, d);
        }
        return (int32_t)pred;
    }
    uint64_t m1[3] = {c[0], c[1], c[2]}, p1[3] = {c[0], c[1], c[2]}, m3[3] = {c[0], c[1], c[2]},
             p3[3] = {c[0], c[1], c[2]};
    m1[a] -= (uint64_t)s;
    p1[a] += (uint64_t)s;
    int has_m3 = c[a] >= (uint64_t)(3 * s), has_p1 = c[a] + s < g->n[a], has_p3 = c[a] + 3 * s < g->n[a];
    if (has_m3 && has_p3) {
        m3[a] -= (uint64_t)(3 * s);
        p3[a] += (uint64_t)(3 * s);
        int64_t num = -(int64_t)qat(g, q, m3) + 9 * (int64_t)qat(g, q, m1) + 9 * (int64_t)qat(g, q, p1) -
                      (int64_t)qat(g, q, p3);
        return (int32_t)floordiv(num + 8, 16);
    }
    if (has_p1) return (int32_t)floordiv((int64_t)qat(g, q, m1) + (int64_t)qat(g, q, p1) + 1, 2);
    return qat(g, q, m1);
}

/* Inverse over the whole field, in place: residuals in, grid values out. */
static void interp_inverse(const geom_t *g, int32_t *a) {
    /* anchors: inclusive prefix sums along each axis of the anchor grid */
    for (int ax = 0; ax < g->ndim; ax++)
        for (uint64_t z = 0; z < g->n[2]; z += (g->ndim >= 3 ? 8 : 1))
            for (uint64_t y = 0; y < g->n[1]; y += (g->ndim >= 2 ? 8 : 1))
                for (uint64_t x = 0; x < g->n[0]; x += 8) {
                    uint64_t c[3] = {x, y, z};
                    if (c[ax] < 8) continue;
                    uint64_t d[3] = {x, y, z};
                    d[ax] -= 8;
                    a[rm(g, x, y, z)] += a[rm(g, d[0], d[1], d[2])];
                }
    /* levels: stride 4, 2, 1; the z-odd, then y-odd, then x-odd points */
    for (int s = 4; s >= 1; s >>= 1)
        for (int ax = g->ndim - 1; ax >= 0; ax--)
            for (uint64_t z = 0; z < g->n[2]; z++)
                for (uint64_t y = 0; y < g->n[1]; y++)
                    for (uint64_t x = 0; x < g->n[0]; x++) {
                        uint64_t c[3] = {x, y, z};
                        int st;
                        if (interp_axis(g, c, &st) != ax || st != s) continue;
                        uint64_t i = rm(g, x, y, z);
                        a[i] = (int32_t)((uint32_t)a[i] + (uint32_t)interp_pred(g, a, x, y, z));
                    }
}

/* ------------------------------------------ global (non-blocked) Lorenzo
 * The first-order Lorenzo predictor of Sec. 3.1 over the whole field: the
 * same formula as P0 with neighbours taken anywhere in the field (zero only
 * outside it), so block faces cost nothing.  Residuals modulo 2^32.  The
 * inverse is the inclusive prefix sum along x of every row of the field,
 * then along y, then along z (the Lorenzo residual is the backward
 * difference along each axis, and prefix sums undo them one axis at a
 * time).  Codes, outliers, patches, chunks and container as for P0; header
 * predictor 6, no map.                                                    */
#define ORC_P_GLOBAL 6

static int32_t gnb(const geom_t *g, const int32_t *q, uint64_t x, uint64_t y, uint64_t z, int dx, int dy, int dz) {
    /* q at (x-dx, y-dy, z-dz) if that point lies in the field, else 0 */
    if ((uint64_t)dx > x || (uint64_t)dy > y || (uint64_t)dz > z) return 0;
    return q[rm(g, x - dx, y - dy, z - dz)];
}

static int32_t global_lorenzo_at(const geom_t *g, const int32_t *q, uint64_t x, uint64_t y, uint64_t z) {
    /* sum over the corners (dx, dy, dz) of the unit cell below the point,
     * sign (-1)^(dx + dy + dz), axes beyond ndim fixed at 0 */
    int64_t d = 0;
    for (int dz = 0; dz <= (g->ndim >= 3); dz++)
        for (int dy = 0; dy <= (g->ndim >= 2); dy++)
            for (int dx = 0; dx <= 1; dx++) {
                int64_t v = gnb(g, q, x, y, z, dx, dy, dz);
                d += ((dx + dy + dz) & 1) ? -v : v;
            }
    return (int32_t)(uint32_t)(uint64_t)d;
}

static void global_inverse(const geom_t *g, int32_t *a) {
    for (int axis = 0; axis < g->ndim; axis++)
        for (uint64_t z = 0; z < g->n[2]; z++)
            for (uint64_t y = 0; y < g->n[1]; y++)
                for (uint64_t x = 0; x < g->n[0]; x++) {
                    uint64_t c[3] = {x, y, z};
                    if (c[axis] == 0) continue;
                    c[axis] -= 1;
                    uint64_t i = rm(g, x, y, z);
                    a[i] = (int32_t)((uint32_t)a[i] + (uint32_t)a[rm(g, c[0], c[1], c[2])]);
                }
}

static int32_t residual_at(const geom_t *g, const int32_t *q, uint64_t x, uint64_t y, uint64_t z, int p,
                           const int32_t coef[4]) {
    if (p == ORC_P1) return lorenzo2_at(g, q, x, y, z);
    if (p == ORC_P_INTERP) return (int32_t)((uint32_t)q[rm(g, x, y, z)] - (uint32_t)interp_pred(g, q, x, y, z));
    if (p == ORC_P_GLOBAL) return global_lorenzo_at(g, q, x, y, z);
    if (p == ORC_P2) {
        int ext[3];
        uint64_t bc[3];
        uint64_t b = (x / g->bs[0]) + g->nb[0] * ((y / g->bs[1]) + g->nb[1] * (z / g->bs[2]));
        block_coords(g, b, bc, ext);
        return q[rm(g, x, y, z)] - regression_pred(coef, ext, (int)(x % g->bs[0]), (int)(y % g->bs[1]),
                                                   (int)(z % g->bs[2]));
    }
    /* P0: backward difference along every axis */
    if (g->ndim == 1) return qnb(g, q, x, y, z, 0, 0, 0) - qnb(g, q, x, y, z, 1, 0, 0);
    if (g->ndim == 2)
        return qnb(g, q, x, y, z, 0, 0, 0) - qnb(g, q, x, y, z, 1, 0, 0) - qnb(g, q, x, y, z, 0, 1, 0) +
               qnb(g, q, x, y, z, 1, 1, 0);
    return qnb(g, q, x, y, z, 0, 0, 0) - qnb(g, q, x, y, z, 1, 0, 0) - qnb(g, q, x, y, z, 0, 1, 0) -
           qnb(g, q, x, y, z, 0, 0, 1) + qnb(g, q, x, y, z, 1, 1, 0) + qnb(g, q, x, y, z, 1, 0, 1) +
           qnb(g, q, x, y, z, 0, 1, 1) - qnb(g, q, x, y, z, 1, 1, 1);
}

/* Inverse for one block, in place on a row-major field: residuals in,
 * grid values out.  P0: inclusive prefix sums along x, then y, then z;
 * P1: the same done twice per axis; P2: add the plane back.              */
static void block_inverse(const geom_t *g, int32_t *a, uint64_t b, int p, const int32_t coef[4]) {
    uint64_t bc[3];
    int ext[3];
    block_coords(g, b, bc, ext);
    uint64_t o[3] = {bc[0] * g->bs[0], bc[1] * g->bs[1], bc[2] * g->bs[2]};
    if (p == ORC_P2) {
        for (int lz = 0; lz < ext[2]; lz++)
            for (int ly = 0; ly < ext[1]; ly++)
                for (int lx = 0; lx < ext[0]; lx++)
                    a[rm(g, o[0] + lx, o[1] + ly, o[2] + lz)] += regression_pred(coef, ext, lx, ly, lz);
        return;
    }
    int passes = (p == ORC_P1) ? 2 : 1;
    for (int axis = 0; axis < 3; axis++)
        for (int rep = 0; rep < passes; rep++)
            for (int lz = 0; lz < ext[2]; lz++)
                for (int ly = 0; ly < ext[1]; ly++)
                    for (int lx = 0; lx < ext[0]; lx++) {
                        int l[3] = {lx, ly, lz};
                        if (l[axis] == 0) continue;
                        int m[3] = {lx, ly, lz};
                        m[axis] -= 1;
                        a[rm(g, o[0] + lx, o[1] + ly, o[2] + lz)] += a[rm(g, o[0] + m[0], o[1] + m[1], o[2] + m[2])];
                    }
}

/* Residual fields for tests: every block with predictor p (P2 coefficients
 * written to coef[4 * nblocks] when coef is not NULL). */
void orc_residual(const int32_t *q, int ndim, const uint64_t dims[3], int p, int32_t *delta, int32_t *coef) {
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return;
    int32_t *cf = (int32_t *)calloc(4 * g.nblocks, sizeof(int32_t));
    if (p == ORC_P2)
        for (uint64_t b = 0; b < g.nblocks; b++) regression_coeffs(&g, q, b, cf + 4 * b);
    for (uint64_t z = 0; z < g.n[2]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[0]; x++) {
                uint64_t b = (x / g.bs[0]) + g.nb[0] * ((y / g.bs[1]) + g.nb[1] * (z / g.bs[2]));
                delta[rm(&g, x, y, z)] = residual_at(&g, q, x, y, z, p, cf + 4 * b);
            }
    if (coef) memcpy(coef, cf, sizeof(int32_t) * 4 * g.nblocks);
    free(cf);
}

void orc_residual_inverse(const int32_t *delta, int ndim, const uint64_t dims[3], int p, const int32_t *coef,
                          int32_t *q) {
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return;
    memcpy(q, delta, sizeof(int32_t) * g.N);
    if (p == ORC_P_INTERP) {
        interp_inverse(&g, q);
        return;
    }
    if (p == ORC_P_GLOBAL) {
        global_inverse(&g, q);
        return;
    }
    for (uint64_t b = 0; b < g.nblocks; b++) block_inverse(&g, q, b, p, coef ? coef + 4 * b : NULL);
}

/* For tests: the interpolation axis of every point (-1 = anchor) and its
 * stride (8 for anchors). */
void orc_interp_classes(int ndim, const uint64_t dims[3], int8_t *axis, uint8_t *stride) {
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return;
    for (uint64_t z = 0; z < g.n[2]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[0]; x++) {
                uint64_t c[3] = {x, y, z};
                int s;
                axis[rm(&g, x, y, z)] = (int8_t)interp_axis(&g, c, &s);
                stride[rm(&g, x, y, z)] = (uint8_t)s;
            }
}

/* ---------------------------------------------------------- container layout
 * header (128 B) | code lengths, 4 bits each, 512 B | [predictor map,
 * 2 bits per block, when the predictor is chosen per block] | [regression
 * coefficients, i32[4] per P2 block in block order] | chunk bits
 * u16[nblocks] | stream u32[words] | outlier pos u32[] | outlier residual
 * i32[] | patch pos u32[] | patch float bits u32[]; every section starts
 * on a 16-byte boundary and padding is zero.  Verbatim container: header
 * with flag bit 0 set, then the raw floats in row-major order.
 * Header predictor field: 0, 1, 2 = P0, P1, P2 for every block; 3 = chosen
 * per block by the learned selector; 4 = chosen per block by exhaustive
 * trial (3 and 4 carry the map).                                          */
typedef struct {
    uint64_t lens, map, coef, chunks, stream, opos, oval, ppos, pbits, total;
} layout_t;

static layout_t make_layout(uint64_t nblocks, int has_map, uint64_t nreg, uint64_t words, uint64_t nout,
                            uint64_t npat) {
    layout_t L;
    L.lens = ORC_HDR;
    L.map = L.lens + ORC_NBINS / 2;
    L.coef = a16(L.map + (has_map ? (nblocks + 3) / 4 : 0));
    L.chunks = a16(L.coef + 16 * nreg);
    L.stream = a16(L.chunks + 2 * nblocks);
    L.opos = a16(L.stream + 4 * words);
    L.oval = a16(L.opos + 4 * nout);
    L.ppos = a16(L.oval + 4 * nout);
    L.pbits = a16(L.ppos + 4 * npat);
    L.total = a16(L.pbits + 4 * npat);
    return L;
}

uint64_t orc_compress_bound(int ndim, const uint64_t dims[3]) {
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return 0;
    return ORC_HDR + 4 * g.N;
}

static void write_header(uint8_t *h, const geom_t *g, int flags, int mode, double eb, double eb_abs,
                         uint64_t total, uint64_t nblocks, uint64_t nout, uint64_t npat,
                         uint64_t words, uint64_t bits, int pred, uint64_t nreg) {
    memset(h, 0, ORC_HDR);
    st32(h + 0, ORC_MAGIC);
    st16(h + 4, ORC_VERSION);
    st16(h + 6, (uint16_t)flags);
    st32(h + 8, (uint32_t)g->ndim);
    st32(h + 12, (uint32_t)pred);
    st64(h + 16, g->n[0]);
    st64(h + 24, g->n[1]);
    st64(h + 32, g->n[2]);
    st32(h + 40, (uint32_t)mode);
    st32(h + 44, ORC_RADIUS);
    st64(h + 48, f64bits(eb));
    st64(h + 56, f64bits(eb_abs));
    st64(h + 64, total);
    st32(h + 72, (uint32_t)nblocks);
    st32(h + 76, (uint32_t)nout);
    st32(h + 80, (uint32_t)npat);
    st32(h + 84, (uint32_t)words);
    st64(h + 88, bits);
    st32(h + 96, (uint32_t)nreg);
}

/* Codes of every value in block-major order for the given per-block
 * predictors; residuals kept for the outlier list; P2 coefficients per
 * block (zero for other blocks). */
static void block_codes(const geom_t *g, const int32_t *q, const elem_ref *refs, const uint8_t *bp,
                        const int32_t *cf, uint16_t *codes, int32_t *res) {
    for (uint64_t k = 0; k < g->N; k++) {
        uint64_t idx = refs[k].idx;
        uint64_t x = idx % g->n[0], y = (idx / g->n[0]) % g->n[1], z = idx / (g->n[0] * g->n[1]);
        uint64_t b = refs[k].pos / ORC_BLOCK_ELEMS;
        int32_t d = residual_at(g, q, x, y, z, bp[b], cf + 4 * b);
        res[k] = d;
        codes[k] = postquant(d);
    }
}

/* ---------------------------------------- exhaustive per-block trial
 * Reference code: the Huffman code of the histogram of P0 codes over the
 * whole field (a code that does not occur there costs 13 bits).  For every
 * block and predictor: cost = sum of reference code lengths + 64 bits per
 * outlier (its position and residual) + 128 bits of coefficients for P2.
 * The block takes the cheapest predictor, ties to the lower index.        */
static void trial_choose(const geom_t *g, const int32_t *q, const elem_ref *refs, const uint32_t *bcount,
                         uint8_t *choice, uint32_t *costs) {
    uint16_t *codes = (uint16_t *)malloc(sizeof(uint16_t) * g->N);
    int32_t *res = (int32_t *)malloc(sizeof(int32_t) * g->N);
    int32_t *cf = (int32_t *)calloc(4 * g->nblocks, sizeof(int32_t));
    uint8_t *bp = (uint8_t *)calloc(g->nblocks, 1);
    uint32_t hist[ORC_NBINS];
    uint8_t len[ORC_NBINS];
    block_codes(g, q, refs, bp, cf, codes, res);
    orc_histogram(codes, g->N, hist);
    orc_codebook(hist, len);
    for (uint64_t b = 0; b < g->nblocks; b++) regression_coeffs(g, q, b, cf + 4 * b);
    uint64_t *cost = (uint64_t *)calloc(3 * g->nblocks, sizeof(uint64_t));
    for (int p = 0; p < 3; p++) {
        memset(bp, p, g->nblocks);
        block_codes(g, q, refs, bp, cf, codes, res);
        uint64_t k = 0;
        for (uint64_t b = 0; b < g->nblocks; b++) {
            uint64_t c = (p == ORC_P2) ? 128 : 0;
            for (uint32_t e = 0; e < bcount[b]; e++, k++) {
                c += len[codes[k]] ? len[codes[k]] : (ORC_LMAX + 1);
                if (codes[k] == 0) c += 64;
            }
            cost[3 * b + p] = c;
        }
    }
    for (uint64_t b = 0; b < g->nblocks; b++) {
        int best = 0;
        for (int p = 1; p < 3; p++)
            if (cost[3 * b + p] < cost[3 * b + best]) best = p;
        choice[b] = (uint8_t)best;
        if (costs)
            for (int p = 0; p < 3; p++) costs[3 * b + p] = (uint32_t)cost[3 * b + p];
    }
    free(codes); free(res); free(cf); free(bp); free(cost);
}

/* ---------------------------------------------------------------- compress
 * pred: 0, 1, 2 = that predictor for every block; 3 = per-block choice
 * given in choice_in (by the learned selector); 4 = per-block choice by
 * exhaustive trial.                                                       */
int orc_compress_ex(const float *x, int ndim, const uint64_t dims[3], int mode, double eb, int pred,
                    const uint8_t *choice_in, uint8_t *out, uint64_t cap, uint64_t *out_bytes) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    if (pred < 0 || pred > 6 || (pred == 3 && !choice_in)) return ORC_ERR_ARG;
    if (cap < ORC_HDR + 4 * g.N) return ORC_ERR_CAPACITY;
    double eb_abs;
    rc = orc_eb_abs(x, g.N, mode, eb, &eb_abs);
    if (rc) return rc;

    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * g.N);
    uint8_t *patch = (uint8_t *)malloc(g.N);
    int32_t *res = (int32_t *)malloc(sizeof(int32_t) * g.N);
    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g.N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g.nblocks);
    uint16_t *codes = (uint16_t *)malloc(sizeof(uint16_t) * g.N);
    uint8_t *bp = (uint8_t *)malloc(g.nblocks);
    int32_t *cf = (int32_t *)calloc(4 * g.nblocks, sizeof(int32_t));
    if (!q || !patch || !res || !refs || !bcount || !codes || !bp || !cf) {
        free(q); free(patch); free(res); free(refs); free(bcount); free(codes); free(bp); free(cf);
        return ORC_ERR_NOMEM;
    }
    orc_prequant(x, g.N, eb_abs, q, patch);
    block_major_order(&g, refs, bcount);
    if (pred <= 2 || pred == ORC_P_INTERP || pred == ORC_P_GLOBAL) memset(bp, pred, g.nblocks);
    else if (pred == 3) memcpy(bp, choice_in, g.nblocks);
    else trial_choose(&g, q, refs, bcount, bp, NULL);
    uint64_t nreg = 0;
    for (uint64_t b = 0; b < g.nblocks; b++) {
        if (bp[b] > ORC_P2 && bp[b] != ORC_P_INTERP && bp[b] != ORC_P_GLOBAL) bp[b] = ORC_P0;
        if (bp[b] == ORC_P2) {
            regression_coeffs(&g, q, b, cf + 4 * b);
            nreg++;
        }
    }
    /* the map costs a quarter byte per block: it is kept only when at
     * least one block in 64 leaves first-order Lorenzo (a switched block
     * then pays for at most 128 bits of map); otherwise every block is
     * coded with first-order Lorenzo in a first-order container */
    if (pred == 3 || pred == 4) {
        uint64_t off = 0;
        for (uint64_t b = 0; b < g.nblocks; b++) off += bp[b] != ORC_P0;
        if (64 * off < g.nblocks) {
            pred = ORC_P0;
            memset(bp, ORC_P0, g.nblocks);
            nreg = 0;
        }
    }
    block_codes(&g, q, refs, bp, cf, codes, res);

    uint64_t nout = 0, npat = 0;
    for (uint64_t k = 0; k < g.N; k++) {
        if (codes[k] == 0) nout++;
        if (patch[refs[k].idx]) npat++;
    }
    uint32_t hist[ORC_NBINS];
    orc_histogram(codes, g.N, hist);
    uint8_t len[ORC_NBINS];
    uint32_t cw[ORC_NBINS];
    orc_codebook(hist, len);
    orc_canonical(len, ORC_NBINS, cw);

    uint64_t bits = 0;
    for (int s = 0; s < ORC_NBINS; s++) bits += (uint64_t)hist[s] * len[s];
    uint64_t words = (bits + 31) / 32;
    int has_map = pred == 3 || pred == 4;
    layout_t L = make_layout(g.nblocks, has_map, nreg, words, nout, npat);

    if (L.total >= ORC_HDR + 4 * g.N) {
        write_header(out, &g, 1, mode, eb, eb_abs, ORC_HDR + 4 * g.N, 0, 0, 0, 0, 0, pred, 0);
        for (uint64_t i = 0; i < g.N; i++) memcpy(out + ORC_HDR + 4 * i, &x[i], 4);
        *out_bytes = ORC_HDR + 4 * g.N;
    } else {
        memset(out, 0, L.total);
        write_header(out, &g, 0, mode, eb, eb_abs, L.total, g.nblocks, nout, npat, words, bits, pred, nreg);
        for (int s = 0; s < ORC_NBINS; s++)
            out[L.lens + s / 2] |= (uint8_t)((len[s] & 15) << (4 * (s % 2)));
        if (has_map)
            for (uint64_t b = 0; b < g.nblocks; b++) out[L.map + b / 4] |= (uint8_t)(bp[b] << (2 * (b % 4)));
        uint64_t ir = 0;
        for (uint64_t b = 0; b < g.nblocks; b++)
            if (bp[b] == ORC_P2) {
                for (int k = 0; k < 4; k++) st32(out + L.coef + 16 * ir + 4 * k, (uint32_t)cf[4 * b + k]);
                ir++;
            }
        uint32_t *stream = (uint32_t *)calloc(words + 1, sizeof(uint32_t));
        bitw bw = {stream, 0};
        uint64_t k = 0, io = 0, ip = 0;
        for (uint64_t b = 0; b < g.nblocks; b++) {
            uint64_t start = bw.nbits;
            for (uint32_t e = 0; e < bcount[b]; e++, k++) {
                put_bits(&bw, cw[codes[k]], len[codes[k]]);
                if (codes[k] == 0) {
                    st32(out + L.opos + 4 * io, refs[k].pos);
                    st32(out + L.oval + 4 * io, (uint32_t)res[k]);
                    io++;
                }
                if (patch[refs[k].idx]) {
                    uint32_t fb;
                    memcpy(&fb, &x[refs[k].idx], 4);
                    st32(out + L.ppos + 4 * ip, refs[k].pos);
                    st32(out + L.pbits + 4 * ip, fb);
                    ip++;
                }
            }
            st16(out + L.chunks + 2 * b, (uint16_t)(bw.nbits - start));
        }
        for (uint64_t w = 0; w < words; w++) st32(out + L.stream + 4 * w, stream[w]);
        free(stream);
        *out_bytes = L.total;
    }
    free(q); free(patch); free(res); free(refs); free(bcount); free(codes); free(bp); free(cf);
    return ORC_OK;
}

int orc_compress(const float *x, int ndim, const uint64_t dims[3], int mode, double eb,
                 uint8_t *out, uint64_t cap, uint64_t *out_bytes) {
    return orc_compress_ex(x, ndim, dims, mode, eb, 0, NULL, out, cap, out_bytes);
}

/* Per-block trial choices (and the three costs per block) for tests and
 * for training labels. */
int orc_trial(const float *x, int ndim, const uint64_t dims[3], int mode, double eb, uint8_t *choice,
              uint32_t *costs) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    double eb_abs;
    rc = orc_eb_abs(x, g.N, mode, eb, &eb_abs);
    if (rc) return rc;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * g.N);
    uint8_t *patch = (uint8_t *)malloc(g.N);
    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g.N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g.nblocks);
    orc_prequant(x, g.N, eb_abs, q, patch);
    block_major_order(&g, refs, bcount);
    trial_choose(&g, q, refs, bcount, choice, costs);
    free(q); free(patch); free(refs); free(bcount);
    return ORC_OK;
}

/* -------------------------------------------------------------- decompress
 * Canonical decoding, one bit at a time: a codeword of length L is the
 * L-bit value v with first[L] <= v < first[L] + count[L]; its symbol is
 * the (v - first[L])-th symbol of length L in symbol order.              */
int orc_header(const uint8_t *in, uint64_t n, int *ndim, uint64_t dims[3], int *mode,
               double *eb, double *eb_abs, int *verbatim) {
    if (n < ORC_HDR) return ORC_ERR_CORRUPT;
    if (ld32(in) != ORC_MAGIC || ld16(in + 4) != ORC_VERSION) return ORC_ERR_CORRUPT;
    *verbatim = ld16(in + 6) & 1;
    *ndim = (int)ld32(in + 8);
    dims[0] = ld64(in + 16);
    dims[1] = ld64(in + 24);
    dims[2] = ld64(in + 32);
    *mode = (int)ld32(in + 40);
    *eb = bitsf64(ld64(in + 48));
    *eb_abs = bitsf64(ld64(in + 56));
    return ORC_OK;
}

static int speed_decompress(const uint8_t *in, const geom_t *g, double eb_abs, float *out);

int orc_decompress(const uint8_t *in, uint64_t n, float *out, uint64_t out_elems) {
    int ndim, mode, verbatim;
    uint64_t dims[3];
    double eb, eb_abs;
    int rc = orc_header(in, n, &ndim, dims, &mode, &eb, &eb_abs, &verbatim);
    if (rc) return rc;
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return ORC_ERR_CORRUPT;
    int pred = (int)ld32(in + 12);
    if (pred > 6 || ld32(in + 44) != ORC_RADIUS) return ORC_ERR_UNSUPPORTED;
    if (out_elems < g.N) return ORC_ERR_CAPACITY;
    uint64_t total = ld64(in + 64);
    if (total > n) return ORC_ERR_CORRUPT;
    if (ld16(in + 6) & ~(1 | ORC_FLAG_SHUFFLE)) return ORC_ERR_CORRUPT;
    if (verbatim) {
        if (total != ORC_HDR + 4 * g.N) return ORC_ERR_CORRUPT;
        memcpy(out, in + ORC_HDR, 4 * g.N);
        return ORC_OK;
    }
    if (ld16(in + 6) & ORC_FLAG_SHUFFLE) return speed_decompress(in, &g, eb_abs, out);
    if (!(eb_abs >= 1e-300 && eb_abs <= 1e300)) return ORC_ERR_CORRUPT;
    uint64_t nblocks = ld32(in + 72), nout = ld32(in + 76), npat = ld32(in + 80);
    uint64_t words = ld32(in + 84), bits = ld64(in + 88), nreg = ld32(in + 96);
    if (nblocks != g.nblocks || words != (bits + 31) / 32) return ORC_ERR_CORRUPT;
    int has_map = pred == 3 || pred == 4;
    if (nreg > g.nblocks) return ORC_ERR_CORRUPT;
    layout_t L = make_layout(nblocks, has_map, nreg, words, nout, npat);
    if (L.total != total) return ORC_ERR_CORRUPT;

    /* per-block predictors and coefficients */
    uint8_t *bp = (uint8_t *)malloc(g.nblocks);
    int32_t *cf = (int32_t *)calloc(4 * g.nblocks, sizeof(int32_t));
    uint64_t ir = 0;
    for (uint64_t b = 0; b < g.nblocks; b++) {
        bp[b] = has_map ? (uint8_t)((in[L.map + b / 4] >> (2 * (b % 4))) & 3) : (uint8_t)pred;
        if (bp[b] > ORC_P2 && bp[b] != ORC_P_INTERP && bp[b] != ORC_P_GLOBAL) { free(bp); free(cf); return ORC_ERR_CORRUPT; }
        if (bp[b] == ORC_P2) {
            if (ir >= nreg) { free(bp); free(cf); return ORC_ERR_CORRUPT; }
            for (int k = 0; k < 4; k++) cf[4 * b + k] = (int32_t)ld32(in + L.coef + 16 * ir + 4 * k);
            ir++;
        }
    }
    if (ir != nreg) { free(bp); free(cf); return ORC_ERR_CORRUPT; }

    uint8_t len[ORC_NBINS];
    for (int s = 0; s < ORC_NBINS; s++) len[s] = (in[L.lens + s / 2] >> (4 * (s % 2))) & 15;
    /* the code must be complete: Kraft sum exactly 1 */
    uint64_t kraft = 0;
    int used = 0;
    for (int s = 0; s < ORC_NBINS; s++) {
        if (len[s] > ORC_LMAX) { free(bp); free(cf); return ORC_ERR_CORRUPT; }
        if (len[s]) { kraft += 1ull << (ORC_LMAX - len[s]); used++; }
    }
    if (used < 2 || kraft != (1ull << ORC_LMAX)) { free(bp); free(cf); return ORC_ERR_CORRUPT; }
    uint32_t first[ORC_LMAX + 2], count[ORC_LMAX + 2];
    static int symidx[ORC_LMAX + 2][ORC_NBINS];
    uint32_t cw[ORC_NBINS];
    orc_canonical(len, ORC_NBINS, cw);
    for (int L2 = 0; L2 <= ORC_LMAX + 1; L2++) { first[L2] = 0xFFFFFFFFu; count[L2] = 0; }
    for (int L2 = 1; L2 <= ORC_LMAX; L2++)
        for (int s = 0; s < ORC_NBINS; s++)
            if (len[s] == L2) {
                if (count[L2] == 0) first[L2] = cw[s];
                symidx[L2][count[L2]++] = s;
            }

    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g.N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g.nblocks);
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * g.N);
    if (!refs || !bcount || !a) {
        free(refs); free(bcount); free(a); free(bp); free(cf);
        return ORC_ERR_NOMEM;
    }
    block_major_order(&g, refs, bcount);
    const uint8_t *stream = in + L.stream;
    uint64_t bitpos = 0, k = 0, io = 0;
    rc = ORC_OK;
    for (uint64_t b = 0; b < g.nblocks && rc == ORC_OK; b++) {
        uint64_t start = bitpos;
        for (uint32_t e = 0; e < bcount[b] && rc == ORC_OK; e++, k++) {
            uint32_t v = 0;
            int L2 = 0, sym = -1;
            while (L2 < ORC_LMAX) {
                if (bitpos >= bits) { rc = ORC_ERR_CORRUPT; break; }
                uint32_t word = ld32(stream + 4 * (bitpos / 32));
                uint32_t bit = (word >> (31 - bitpos % 32)) & 1u;
                bitpos++;
                v = (v << 1) | bit;
                L2++;
                if (count[L2] && v >= first[L2] && v - first[L2] < count[L2]) {
                    sym = symidx[L2][v - first[L2]];
                    break;
                }
            }
            if (rc) break;
            if (sym < 0) { rc = ORC_ERR_CORRUPT; break; }
            int32_t d;
            if (sym == 0) {
                if (io >= nout || ld32(in + L.opos + 4 * io) != refs[k].pos) { rc = ORC_ERR_CORRUPT; break; }
                d = (int32_t)ld32(in + L.oval + 4 * io);
                io++;
            } else {
                d = sym - ORC_RADIUS;
            }
            a[refs[k].idx] = d;
        }
        if (rc == ORC_OK && bitpos - start != ld16(in + L.chunks + 2 * b)) rc = ORC_ERR_CORRUPT;
    }
    if (rc == ORC_OK && (io != nout || bitpos != bits)) rc = ORC_ERR_CORRUPT;
    if (rc == ORC_OK) {
        if (pred == ORC_P_INTERP) interp_inverse(&g, a);
        else if (pred == ORC_P_GLOBAL) global_inverse(&g, a);
        else
            for (uint64_t b = 0; b < g.nblocks; b++) block_inverse(&g, a, b, bp[b], cf + 4 * b);
        double e2 = 2.0 * eb_abs;
        for (uint64_t i = 0; i < g.N; i++) out[i] = dequant(a[i], e2);
        /* lossless patches: positions ascending, each names a real element */
        uint64_t kk = 0;
        uint32_t last = 0;
        for (uint64_t ip = 0; ip < npat; ip++) {
            uint32_t pos = ld32(in + L.ppos + 4 * ip);
            uint32_t fb = ld32(in + L.pbits + 4 * ip);
            if (ip > 0 && pos <= last) { rc = ORC_ERR_CORRUPT; break; }
            last = pos;
            while (kk < g.N && refs[kk].pos < pos) kk++;
            if (kk >= g.N || refs[kk].pos != pos) { rc = ORC_ERR_CORRUPT; break; }
            memcpy(&out[refs[kk].idx], &fb, 4);
        }
    }
    free(refs); free(bcount); free(a); free(bp); free(cf);
    return rc;
}

/* ------------------------------------------ bit-shuffle codec (FZMod-Speed)
 * The throughput-oriented pipeline of the paper swaps the Huffman stage
 * for the bit-shuffle and dictionary (zero-word) encoding of FZ-GPU
 * (Sec. 3.2 module list, Sec. 3.3 FZMod-Speed); the paper gives no
 * bit-level detail, so this is the reading the project fixes:
 *   - steps 1-4 as above with first-order Lorenzo in every block;
 *   - every value gets a 10-bit symbol: the residual d (|d| < radius) folded
 *     to an unsigned number, zigzag(d) = 2d for d >= 0 and -2d - 1 for
 *     d < 0 (0, -1, 1, -2, ... -> 0, 1, 2, 3, ...), and 1023 for an outlier;
 *   - a block owns 512 symbol slots (slot = position mod 512; slots of a
 *     truncated block that hold no value are 0), cut into 16 groups of 32;
 *   - bit-shuffle: group g gives 10 words, word p holding bit p of the
 *     group's 32 symbols, symbol j of the group in bit j;
 *   - zero-word elimination: bit 10 g + p of the block's 160-bit mask says
 *     whether word p of group g is non-zero; only non-zero words are kept,
 *     in mask-bit order, blocks one after the other.
 * Container: header (flag bit 1 set, predictor 0, "words" = kept words,
 * "bits" = 0) | masks u32[5 per block] (mask bit k in word k/32, bit k%32)
 * | kept words u32[] | outlier pos u32[] | outlier residual i32[] | patch
 * pos u32[] | patch bits u32[]; sections 16-byte aligned, padding zero.   */
#define ORC_SYM_OUTLIER 1023u
#define ORC_GROUPS 16
#define ORC_PLANES 10
#define ORC_MASK_WORDS 5

typedef struct {
    uint64_t masks, words, opos, oval, ppos, pbits, total;
} slayout_t;

static slayout_t speed_layout(uint64_t nblocks, uint64_t words, uint64_t nout, uint64_t npat) {
    slayout_t L;
    L.masks = ORC_HDR;
    L.words = a16(L.masks + 4 * ORC_MASK_WORDS * nblocks);
    L.opos = a16(L.words + 4 * words);
    L.oval = a16(L.opos + 4 * nout);
    L.ppos = a16(L.oval + 4 * nout);
    L.pbits = a16(L.ppos + 4 * npat);
    L.total = a16(L.pbits + 4 * npat);
    return L;
}

static uint32_t zigzag(int32_t d) { return d >= 0 ? 2u * (uint32_t)d : 2u * (uint32_t)(-(int64_t)d) - 1u; }
static int32_t unzigzag(uint32_t s) { return (s & 1u) ? -(int32_t)((s + 1u) / 2u) : (int32_t)(s / 2u); }

/* Symbols of every block, 512 slots each (block order), from the residual
 * codes: code 0 (outlier) -> 1023, code c -> zigzag(c - radius).          */
static void speed_symbols(const geom_t *g, const elem_ref *refs, const uint16_t *codes, uint16_t *sym) {
    memset(sym, 0, sizeof(uint16_t) * g->nblocks * ORC_BLOCK_ELEMS);
    for (uint64_t k = 0; k < g->N; k++)
        sym[refs[k].pos] = codes[k] == 0 ? (uint16_t)ORC_SYM_OUTLIER : (uint16_t)zigzag((int32_t)codes[k] - ORC_RADIUS);
}

/* word p of one group of 32 symbols */
static uint32_t shuffle_word(const uint16_t *s32, int p) {
    uint32_t w = 0;
    for (int j = 0; j < 32; j++) w |= (uint32_t)((s32[j] >> p) & 1u) << j;
    return w;
}

/* For tests: the symbols (nblocks * 512) and the shuffled words
 * (nblocks * 160, group-major) of a field. */
int orc_speed_stage(const float *x, int ndim, const uint64_t dims[3], int mode, double eb, uint16_t *sym_out,
                    uint32_t *words_out) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    double eb_abs;
    rc = orc_eb_abs(x, g.N, mode, eb, &eb_abs);
    if (rc) return rc;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * g.N);
    uint8_t *patch = (uint8_t *)malloc(g.N);
    int32_t *res = (int32_t *)malloc(sizeof(int32_t) * g.N);
    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g.N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g.nblocks);
    uint16_t *codes = (uint16_t *)malloc(sizeof(uint16_t) * g.N);
    uint8_t *bp = (uint8_t *)calloc(g.nblocks, 1);
    int32_t *cf = (int32_t *)calloc(4 * g.nblocks, sizeof(int32_t));
    orc_prequant(x, g.N, eb_abs, q, patch);
    block_major_order(&g, refs, bcount);
    block_codes(&g, q, refs, bp, cf, codes, res);
    speed_symbols(&g, refs, codes, sym_out);
    for (uint64_t b = 0; b < g.nblocks; b++)
        for (int gi = 0; gi < ORC_GROUPS; gi++)
            for (int p = 0; p < ORC_PLANES; p++)
                words_out[(b * ORC_GROUPS + gi) * ORC_PLANES + p] =
                    shuffle_word(sym_out + b * ORC_BLOCK_ELEMS + 32 * gi, p);
    free(q); free(patch); free(res); free(refs); free(bcount); free(codes); free(bp); free(cf);
    return ORC_OK;
}

int orc_speed_compress(const float *x, int ndim, const uint64_t dims[3], int mode, double eb, uint8_t *out,
                       uint64_t cap, uint64_t *out_bytes) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    if (cap < ORC_HDR + 4 * g.N) return ORC_ERR_CAPACITY;
    double eb_abs;
    rc = orc_eb_abs(x, g.N, mode, eb, &eb_abs);
    if (rc) return rc;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * g.N);
    uint8_t *patch = (uint8_t *)malloc(g.N);
    int32_t *res = (int32_t *)malloc(sizeof(int32_t) * g.N);
    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g.N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g.nblocks);
    uint16_t *codes = (uint16_t *)malloc(sizeof(uint16_t) * g.N);
    uint8_t *bp = (uint8_t *)calloc(g.nblocks, 1);
    int32_t *cf = (int32_t *)calloc(4 * g.nblocks, sizeof(int32_t));
    uint16_t *sym = (uint16_t *)malloc(sizeof(uint16_t) * g.nblocks * ORC_BLOCK_ELEMS);
    uint32_t *mask = (uint32_t *)calloc(ORC_MASK_WORDS * g.nblocks, sizeof(uint32_t));
    uint32_t *kept = (uint32_t *)malloc(sizeof(uint32_t) * (g.nblocks * ORC_GROUPS * ORC_PLANES + 1));
    if (!q || !patch || !res || !refs || !bcount || !codes || !bp || !cf || !sym || !mask || !kept) {
        free(q); free(patch); free(res); free(refs); free(bcount); free(codes); free(bp); free(cf);
        free(sym); free(mask); free(kept);
        return ORC_ERR_NOMEM;
    }
    orc_prequant(x, g.N, eb_abs, q, patch);
    block_major_order(&g, refs, bcount);
    block_codes(&g, q, refs, bp, cf, codes, res);
    speed_symbols(&g, refs, codes, sym);
    /* shuffle and keep the non-zero words */
    uint64_t words = 0;
    for (uint64_t b = 0; b < g.nblocks; b++)
        for (int gi = 0; gi < ORC_GROUPS; gi++)
            for (int p = 0; p < ORC_PLANES; p++) {
                uint32_t w = shuffle_word(sym + b * ORC_BLOCK_ELEMS + 32 * gi, p);
                if (w) {
                    int k = gi * ORC_PLANES + p;
                    mask[ORC_MASK_WORDS * b + k / 32] |= 1u << (k % 32);
                    kept[words++] = w;
                }
            }
    uint64_t nout = 0, npat = 0;
    for (uint64_t k = 0; k < g.N; k++) {
        if (codes[k] == 0) nout++;
        if (patch[refs[k].idx]) npat++;
    }
    slayout_t L = speed_layout(g.nblocks, words, nout, npat);
    if (L.total >= ORC_HDR + 4 * g.N) {
        write_header(out, &g, 1 | ORC_FLAG_SHUFFLE, mode, eb, eb_abs, ORC_HDR + 4 * g.N, 0, 0, 0, 0, 0, 0, 0);
        for (uint64_t i = 0; i < g.N; i++) memcpy(out + ORC_HDR + 4 * i, &x[i], 4);
        *out_bytes = ORC_HDR + 4 * g.N;
    } else {
        memset(out, 0, L.total);
        write_header(out, &g, ORC_FLAG_SHUFFLE, mode, eb, eb_abs, L.total, g.nblocks, nout, npat, words, 0, 0, 0);
        for (uint64_t i = 0; i < ORC_MASK_WORDS * g.nblocks; i++) st32(out + L.masks + 4 * i, mask[i]);
        for (uint64_t i = 0; i < words; i++) st32(out + L.words + 4 * i, kept[i]);
        uint64_t io = 0, ip = 0;
        for (uint64_t k = 0; k < g.N; k++) {
            if (codes[k] == 0) {
                st32(out + L.opos + 4 * io, refs[k].pos);
                st32(out + L.oval + 4 * io, (uint32_t)res[k]);
                io++;
            }
            if (patch[refs[k].idx]) {
                uint32_t fb;
                memcpy(&fb, &x[refs[k].idx], 4);
                st32(out + L.ppos + 4 * ip, refs[k].pos);
                st32(out + L.pbits + 4 * ip, fb);
                ip++;
            }
        }
        *out_bytes = L.total;
    }
    free(q); free(patch); free(res); free(refs); free(bcount); free(codes); free(bp); free(cf);
    free(sym); free(mask); free(kept);
    return ORC_OK;
}

/* Decoding of a bit-shuffle container (header already checked for magic,
 * geometry, size and the verbatim flag by orc_decompress). */
static int speed_decompress(const uint8_t *in, const geom_t *g, double eb_abs, float *out) {
    uint64_t nblocks = ld32(in + 72), nout = ld32(in + 76), npat = ld32(in + 80);
    uint64_t words = ld32(in + 84), total = ld64(in + 64);
    if (nblocks != g->nblocks || ld64(in + 88) != 0 || ld32(in + 12) != ORC_P0 || ld32(in + 96) != 0)
        return ORC_ERR_CORRUPT;
    if (!(eb_abs >= 1e-300 && eb_abs <= 1e300)) return ORC_ERR_CORRUPT;
    slayout_t L = speed_layout(nblocks, words, nout, npat);
    if (L.total != total) return ORC_ERR_CORRUPT;
    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g->N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g->nblocks);
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * g->N);
    uint16_t *sym = (uint16_t *)calloc(g->nblocks * ORC_BLOCK_ELEMS, sizeof(uint16_t));
    if (!refs || !bcount || !a || !sym) {
        free(refs); free(bcount); free(a); free(sym);
        return ORC_ERR_NOMEM;
    }
    block_major_order(g, refs, bcount);
    /* unshuffle: the kept words, in mask-bit order, block after block */
    uint64_t next = 0;
    int rc = ORC_OK;
    for (uint64_t b = 0; b < g->nblocks && rc == ORC_OK; b++)
        for (int k = 0; k < ORC_GROUPS * ORC_PLANES; k++) {
            uint32_t m = ld32(in + L.masks + 4 * (ORC_MASK_WORDS * b + k / 32));
            if (!((m >> (k % 32)) & 1u)) continue;
            if (next >= words) { rc = ORC_ERR_CORRUPT; break; }
            uint32_t w = ld32(in + L.words + 4 * next);
            next++;
            int gi = k / ORC_PLANES, p = k % ORC_PLANES;
            for (int j = 0; j < 32; j++)
                sym[b * ORC_BLOCK_ELEMS + 32 * gi + j] |= (uint16_t)(((w >> j) & 1u) << p);
        }
    /* every kept word used */
    if (rc == ORC_OK && next != words) rc = ORC_ERR_CORRUPT;
    /* residuals; an outlier symbol takes the next listed outlier, whose
     * position must be this value's */
    uint64_t io = 0;
    for (uint64_t k = 0; k < g->N && rc == ORC_OK; k++) {
        uint32_t s = sym[refs[k].pos];
        int32_t d;
        if (s == ORC_SYM_OUTLIER) {
            if (io >= nout || ld32(in + L.opos + 4 * io) != refs[k].pos) { rc = ORC_ERR_CORRUPT; break; }
            d = (int32_t)ld32(in + L.oval + 4 * io);
            io++;
        } else {
            d = unzigzag(s);
        }
        a[refs[k].idx] = d;
    }
    if (rc == ORC_OK && io != nout) rc = ORC_ERR_CORRUPT;
    if (rc == ORC_OK) {
        for (uint64_t b = 0; b < g->nblocks; b++) block_inverse(g, a, b, ORC_P0, NULL);
        double e2 = 2.0 * eb_abs;
        for (uint64_t i = 0; i < g->N; i++) out[i] = dequant(a[i], e2);
        uint64_t kk = 0;
        uint32_t last = 0;
        for (uint64_t ip = 0; ip < npat; ip++) {
            uint32_t pos = ld32(in + L.ppos + 4 * ip);
            uint32_t fb = ld32(in + L.pbits + 4 * ip);
            if (ip > 0 && pos <= last) { rc = ORC_ERR_CORRUPT; break; }
            last = pos;
            while (kk < g->N && refs[kk].pos < pos) kk++;
            if (kk >= g->N || refs[kk].pos != pos) { rc = ORC_ERR_CORRUPT; break; }
            memcpy(&out[refs[kk].idx], &fb, 4);
        }
    }
    free(refs); free(bcount); free(a); free(sym);
    return rc;
}

/* ------------------------------------------------------- stage dumps (tests)
 * Codes, outlier count and histogram exactly as compression computes them,
 * in block-major order, for stage-level comparisons.                      */
int orc_stage_codes(const float *x, int ndim, const uint64_t dims[3], int mode, double eb,
                    uint16_t *codes_out, uint32_t *pos_out, uint32_t *hist_out, double *eb_abs_out) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    double eb_abs;
    rc = orc_eb_abs(x, g.N, mode, eb, &eb_abs);
    if (rc) return rc;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * g.N);
    uint8_t *patch = (uint8_t *)malloc(g.N);
    int32_t *delta = (int32_t *)malloc(sizeof(int32_t) * g.N);
    elem_ref *refs = (elem_ref *)malloc(sizeof(elem_ref) * g.N);
    uint32_t *bcount = (uint32_t *)malloc(sizeof(uint32_t) * g.nblocks);
    orc_prequant(x, g.N, eb_abs, q, patch);
    orc_lorenzo1(q, ndim, dims, delta);
    block_major_order(&g, refs, bcount);
    for (uint64_t k = 0; k < g.N; k++) {
        codes_out[k] = postquant(delta[refs[k].idx]);
        if (pos_out) pos_out[k] = refs[k].pos;
    }
    orc_histogram(codes_out, g.N, hist_out);
    *eb_abs_out = eb_abs;
    free(q); free(patch); free(delta); free(refs); free(bcount);
    return ORC_OK;
}

/* Encode a plain symbol sequence with the canonical code of len[] (tests). */
uint64_t orc_encode_symbols(const uint16_t *syms, uint64_t n, const uint8_t *len, int nsym, uint32_t *words) {
    uint32_t *cw = (uint32_t *)malloc(sizeof(uint32_t) * nsym);
    orc_canonical(len, nsym, cw);
    bitw bw = {words, 0};
    for (uint64_t i = 0; i < n; i++) put_bits(&bw, cw[syms[i]], len[syms[i]]);
    free(cw);
    return bw.nbits;
}

/* ------------------------------------------------ block features
 * Sixteen statistics of a sample of each block's prequantised values q,
 * the input of the learned predictor selector.  The paper leaves automatic
 * predictor choice to future work (Sec. 5); this feature set (version 2)
 * is this project's reading.  The sample is the block's first
 * ORC_FSAMPLE = 128 positions in its row-major order (the two lowest
 * z-planes of a 3D block, the four lowest rows of a 2D block, the first
 * 128 values of a 1D block), real points only: a lower box of the block,
 * so every neighbour a statistic below uses is in the sample or outside
 * the block.  Only quantities cheaper than the predictors themselves (no
 * second-order stencil, no regression fit), so that choosing costs less
 * than trying.  Every feature is built from
 * exact integer sums with the same IEEE operations on any machine: one
 * double division, rounding to float, then plog2(1 + v), the
 * piecewise-linear base-2 logarithm read from the float's bits (integer
 * subtraction, one int-to-float rounding, a multiplication by 2^-23).
 *   0      plog2(1 + variance of q)
 *   1      plog2(1 + max q - min q)
 *   2, 3, 4   plog2(1 + mean |first difference|) along x, y, z
 *   5, 6, 7   plog2(1 + mean |second difference|) along x, y, z
 *   8, 9, 10  plog2(1 + mean |mixed difference|) in xy, yz, xz
 *   11     plog2(1 + mean |first-order Lorenzo residual|)
 *   12     plog2(1 + max |first-order Lorenzo residual|)
 *   13     fraction of first-order residuals outside the code range
 *   14     plog2(1 + max |q|)
 *   15     plog2(1 + |mean of q|)
 * Differences use point pairs (triples) inside the sample; a mean over no
 * pairs is 0.  Lorenzo residuals take neighbours outside the block as 0,
 * exactly as the predictors do.                                          */
#define ORC_NFEAT 16
#define ORC_FSAMPLE 128

static float plog2_1p(double v) {
    float f = (float)v;
    float a = 1.0f + f;
    uint32_t u;
    memcpy(&u, &a, 4);
    return (float)(int32_t)(u - 0x3F800000u) * (1.0f / 8388608.0f);
}

static double mean_of(int64_t s, int64_t n) { return n > 0 ? (double)s / (double)n : 0.0; }

static void block_features(const geom_t *g, const int32_t *q, uint64_t b, float *f) {
    uint64_t bc[3];
    int ext[3];
    block_coords(g, b, bc, ext);
    /* the sample: the lower box holding the first ORC_FSAMPLE row-major
     * positions of the block */
    {
        int a = g->ndim - 1;
        int span = 1;
        for (int k = 0; k < a; k++) span *= (int)g->bs[k];
        int lim = ORC_FSAMPLE / span;
        if (ext[a] > lim) ext[a] = lim;
    }
    uint64_t o[3] = {bc[0] * g->bs[0], bc[1] * g->bs[1], bc[2] * g->bs[2]};
    int64_t n = (int64_t)ext[0] * ext[1] * ext[2];
    int64_t s1 = 0, s2 = 0, lo = INT64_MAX, hi = INT64_MIN;
    int64_t d1[3] = {0, 0, 0}, c1[3] = {0, 0, 0}, d2[3] = {0, 0, 0}, c2[3] = {0, 0, 0};
    int64_t dm[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
    int64_t r0 = 0, r0max = 0, nout = 0;
    const int32_t coef[4] = {0, 0, 0, 0};  /* the first-order residual uses none */
#define Q(lx, ly, lz) ((int64_t)q[rm(g, o[0] + (lx), o[1] + (ly), o[2] + (lz))])
    for (int lz = 0; lz < ext[2]; lz++)
        for (int ly = 0; ly < ext[1]; ly++)
            for (int lx = 0; lx < ext[0]; lx++) {
                int64_t v = Q(lx, ly, lz);
                int l[3] = {lx, ly, lz};
                s1 += v;
                s2 += v * v;
                if (v < lo) lo = v;
                if (v > hi) hi = v;
                for (int a = 0; a < 3; a++) {
                    int e[3] = {0, 0, 0};
                    e[a] = 1;
                    if (l[a] >= 1) {
                        d1[a] += llabs(v - Q(lx - e[0], ly - e[1], lz - e[2]));
                        c1[a]++;
                    }
                    if (l[a] >= 2) {
                        d2[a] += llabs(v - 2 * Q(lx - e[0], ly - e[1], lz - e[2]) +
                                       Q(lx - 2 * e[0], ly - 2 * e[1], lz - 2 * e[2]));
                        c2[a]++;
                    }
                }
                /* mixed differences: xy, yz, xz */
                int pa[3][2] = {{0, 1}, {1, 2}, {0, 2}};
                for (int m = 0; m < 3; m++) {
                    int a0 = pa[m][0], a1 = pa[m][1];
                    if (l[a0] >= 1 && l[a1] >= 1) {
                        int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
                        e0[a0] = 1;
                        e1[a1] = 1;
                        dm[m] += llabs(v - Q(lx - e0[0], ly - e0[1], lz - e0[2]) -
                                       Q(lx - e1[0], ly - e1[1], lz - e1[2]) +
                                       Q(lx - e0[0] - e1[0], ly - e0[1] - e1[1], lz - e0[2] - e1[2]));
                        cm[m]++;
                    }
                }
                uint64_t x = o[0] + lx, y = o[1] + ly, z = o[2] + lz;
                int64_t d0 = residual_at(g, q, x, y, z, ORC_P0, coef);
                int64_t ad0 = llabs(d0);
                r0 += ad0;
                if (ad0 > r0max) r0max = ad0;
                if (d0 <= -ORC_RADIUS || d0 >= ORC_RADIUS) nout++;
            }
#undef Q
    double m = (double)s1 / (double)n;
    double var = (double)s2 / (double)n - m * m;
    if (var < 0.0) var = 0.0;
    f[0] = plog2_1p(var);
    f[1] = plog2_1p((double)(hi - lo));
    for (int a = 0; a < 3; a++) {
        f[2 + a] = plog2_1p(mean_of(d1[a], c1[a]));
        f[5 + a] = plog2_1p(mean_of(d2[a], c2[a]));
        f[8 + a] = plog2_1p(mean_of(dm[a], cm[a]));
    }
    f[11] = plog2_1p(mean_of(r0, n));
    f[12] = plog2_1p((double)r0max);
    f[13] = (float)((double)nout / (double)n);
    f[14] = plog2_1p((double)(llabs(lo) > llabs(hi) ? llabs(lo) : llabs(hi)));
    f[15] = plog2_1p(fabs(m));
}

/* Features of every block (block order), f[16 * nblocks]. */
int orc_features(const float *x, int ndim, const uint64_t dims[3], int mode, double eb, float *feat) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    double eb_abs;
    rc = orc_eb_abs(x, g.N, mode, eb, &eb_abs);
    if (rc) return rc;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * g.N);
    uint8_t *patch = (uint8_t *)malloc(g.N);
    if (!q || !patch) { free(q); free(patch); return ORC_ERR_NOMEM; }
    orc_prequant(x, g.N, eb_abs, q, patch);
    for (uint64_t b = 0; b < g.nblocks; b++) block_features(&g, q, b, feat + ORC_NFEAT * b);
    free(q);
    free(patch);
    return ORC_OK;
}

/* Same, from a grid-value field q (tests). */
int orc_features_q(const int32_t *q, int ndim, const uint64_t dims[3], float *feat) {
    geom_t g;
    int rc = make_geom(ndim, dims, &g);
    if (rc) return rc;
    for (uint64_t b = 0; b < g.nblocks; b++) block_features(&g, q, b, feat + ORC_NFEAT * b);
    return ORC_OK;
}

/* ------------------------------------------------ selector network
 * A multilayer perceptron 16 -> 64 -> 64 -> 3 with ReLU hidden layers
 * predicts log2(1 + bits) of each predictor for a block from its
 * standardised features; the block takes the predictor with the smallest
 * prediction, ties to the lower index.  Parameter vector (floats, in this
 * order): mu[16], rs[16] (standardisation z = (f - mu) * rs), W1[64][16],
 * b1[64], W2[64][64], b2[64], W3[3][64], b3[3].
 * Inference is in float: each dot product is a chain of fused
 * multiply-adds (one rounding per term, IEEE 754-2008 fusedMultiplyAdd,
 * C99 fmaf) in index order starting from the bias, so that any IEEE
 * machine gets the same bits.            */
#define ORC_H 64
#define ORC_NOUT 3
#define OFF_MU 0
#define OFF_RS (OFF_MU + ORC_NFEAT)
#define OFF_W1 (OFF_RS + ORC_NFEAT)
#define OFF_B1 (OFF_W1 + ORC_H * ORC_NFEAT)
#define OFF_W2 (OFF_B1 + ORC_H)
#define OFF_B2 (OFF_W2 + ORC_H * ORC_H)
#define OFF_W3 (OFF_B2 + ORC_H)
#define OFF_B3 (OFF_W3 + ORC_NOUT * ORC_H)
#define ORC_NPARAM (OFF_B3 + ORC_NOUT)

#define ORC_MARGIN 0.0078125f

int orc_mlp_nparam(void) { return ORC_NPARAM; }

void orc_mlp_infer(const float *w, const float *feat, uint64_t n, float *y, uint8_t *choice) {
    for (uint64_t s = 0; s < n; s++) {
        const float *f = feat + ORC_NFEAT * s;
        float z[ORC_NFEAT], h1[ORC_H], h2[ORC_H], o[ORC_NOUT];
        for (int i = 0; i < ORC_NFEAT; i++) {
            float d = f[i] - w[OFF_MU + i];
            z[i] = d * w[OFF_RS + i];
        }
        for (int j = 0; j < ORC_H; j++) {
            float acc = w[OFF_B1 + j];
            for (int i = 0; i < ORC_NFEAT; i++) acc = fmaf(w[OFF_W1 + ORC_NFEAT * j + i], z[i], acc);
            h1[j] = acc > 0.0f ? acc : 0.0f;
        }
        for (int j = 0; j < ORC_H; j++) {
            float acc = w[OFF_B2 + j];
            for (int i = 0; i < ORC_H; i++) acc = fmaf(w[OFF_W2 + ORC_H * j + i], h1[i], acc);
            h2[j] = acc > 0.0f ? acc : 0.0f;
        }
        for (int k = 0; k < ORC_NOUT; k++) {
            float acc = w[OFF_B3 + k];
            for (int i = 0; i < ORC_H; i++) acc = fmaf(w[OFF_W3 + ORC_H * k + i], h2[i], acc);
            o[k] = acc;
        }
        /* the choice: the lowest score, ties to the lower index; a
         * predictor other than first-order Lorenzo scores its output plus
         * ORC_MARGIN = 1/128 (a predicted saving below 2^(1/128) - 1 = 0.54%
         * is not worth the risk of a wrong switch and its share of the
         * map) */
        int best = 0;
        float bs = o[0];
        for (int k = 1; k < ORC_NOUT; k++) {
            float sk = o[k] + ORC_MARGIN;
            if (sk < bs) { best = k; bs = sk; }
        }
        if (y)
            for (int k = 0; k < ORC_NOUT; k++) y[ORC_NOUT * s + k] = o[k];
        if (choice) choice[s] = (uint8_t)best;
    }
}

/* Mean squared error over n samples and the three outputs, and its
 * gradient with respect to every parameter (mu and rs get 0: they are set
 * from the training features, not learned), in double by plain
 * backpropagation:
 *   L = 1 / (3 n) * sum_s sum_k (y_sk - t_sk)^2
 *   dL/dy = 2 (y - t) / (3 n); dL/dW = delta^T * activations; ReLU passes
 *   the gradient where its input is > 0.                                 */
double orc_mlp_loss_grad(const double *w, const float *feat, const double *target, uint64_t n, double *grad) {
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * ORC_NPARAM);
    for (uint64_t s = 0; s < n; s++) {
        const float *f = feat + ORC_NFEAT * s;
        double z[ORC_NFEAT], a1[ORC_H], h1[ORC_H], a2[ORC_H], h2[ORC_H], dy[ORC_NOUT];
        double dh2[ORC_H], dh1[ORC_H];
        for (int i = 0; i < ORC_NFEAT; i++) z[i] = ((double)f[i] - w[OFF_MU + i]) * w[OFF_RS + i];
        for (int j = 0; j < ORC_H; j++) {
            double acc = w[OFF_B1 + j];
            for (int i = 0; i < ORC_NFEAT; i++) acc += w[OFF_W1 + ORC_NFEAT * j + i] * z[i];
            a1[j] = acc;
            h1[j] = acc > 0.0 ? acc : 0.0;
        }
        for (int j = 0; j < ORC_H; j++) {
            double acc = w[OFF_B2 + j];
            for (int i = 0; i < ORC_H; i++) acc += w[OFF_W2 + ORC_H * j + i] * h1[i];
            a2[j] = acc;
            h2[j] = acc > 0.0 ? acc : 0.0;
        }
        for (int k = 0; k < ORC_NOUT; k++) {
            double acc = w[OFF_B3 + k];
            for (int i = 0; i < ORC_H; i++) acc += w[OFF_W3 + ORC_H * k + i] * h2[i];
            double e = acc - target[ORC_NOUT * s + k];
            loss += e * e;
            dy[k] = 2.0 * e / (3.0 * (double)n);
        }
        if (!grad) continue;
        for (int k = 0; k < ORC_NOUT; k++) {
            grad[OFF_B3 + k] += dy[k];
            for (int i = 0; i < ORC_H; i++) grad[OFF_W3 + ORC_H * k + i] += dy[k] * h2[i];
        }
        for (int i = 0; i < ORC_H; i++) {
            double acc = 0.0;
            for (int k = 0; k < ORC_NOUT; k++) acc += dy[k] * w[OFF_W3 + ORC_H * k + i];
            dh2[i] = a2[i] > 0.0 ? acc : 0.0;
        }
        for (int j = 0; j < ORC_H; j++) {
            grad[OFF_B2 + j] += dh2[j];
            for (int i = 0; i < ORC_H; i++) grad[OFF_W2 + ORC_H * j + i] += dh2[j] * h1[i];
        }
        for (int i = 0; i < ORC_H; i++) {
            double acc = 0.0;
            for (int j = 0; j < ORC_H; j++) acc += dh2[j] * w[OFF_W2 + ORC_H * j + i];
            dh1[i] = a1[i] > 0.0 ? acc : 0.0;
        }
        for (int j = 0; j < ORC_H; j++) {
            grad[OFF_B1 + j] += dh1[j];
            for (int i = 0; i < ORC_NFEAT; i++) grad[OFF_W1 + ORC_NFEAT * j + i] += dh1[j] * z[i];
        }
    }
    return loss / (3.0 * (double)n);
}

/* One Adam step (Kingma and Ba) on the learned parameters (W1 onwards),
 * step number t >= 1:
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2
 *   w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)           */
void orc_adam_step(double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                   double eps) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = OFF_W1; i < ORC_NPARAM; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
