/*
 * lbpf_ref.c -- CPU oracle for the depth-fused LBP face-recognition path of
 * Naik & Rathna, "Robust real time face recognition and tracking on GPU using
 * fusion of RGB and depth image" (arXiv 1504.01883).
 *
 * TEST INFRASTRUCTURE. This file is the plain, slow, obviously-correct
 * definition of what the GPU path computes. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it. It shares no source,
 * header, table or constant with the GPU library: the neighbour order, the
 * uniform-pattern table and the cell geometry are all rebuilt here from their
 * definitions.
 *
 * What each function follows:
 *   lbpf_ref_median        -- depth "fusion" region of interest (Sec. 1 and the
 *                             abstract: depth reduces cost and removes pose and
 *                             illumination effects); reading: the lower median
 *                             of the non-zero depth of the crop.
 *   lbpf_ref_lbp_code      -- Sec. 2.4, Eq. 2 and Fig. 7: threshold the eight
 *                             3x3 neighbours against the centre (s(x)=1 iff
 *                             x>=0) and weight neighbour p by 2^p.
 *   lbpf_ref_uniform_bin   -- uniform patterns (Ojala, the paper's ref. [16]):
 *                             at most two 0/1 transitions around the circle.
 *   lbpf_ref_features      -- Sec. 2.4, Eq. 3: per-region histograms of the
 *                             codes, concatenated; Sec. 3: grey (u8) and
 *                             ushort depth images.
 *   lbpf_ref_features_warped -- Sec. 2.1, Eq. 1 (p' = x u + y v + t: the
 *                             affine frame that turns the mapped face region
 *                             into a rectangle) and Sec. 3 (the face resized to
 *                             200 x 200): every crop pixel is sampled from its
 *                             plane through a fixed-point affine frame (nearest
 *                             sample), then the crop goes through
 *                             lbpf_ref_features unchanged.
 *   lbpf_ref_track         -- Sec. 2.3 and Fig. 4: a face is followed into the
 *                             next frame by the detection whose box centre is
 *                             nearest to its centre in the previous frame.
 *   lbpf_ref_score_f64     -- Sec. 2.5: one linear SVM hyperplane per person,
 *                             decision value w.x + b, best score wins.
 *   lbpf_ref_train_ovr_f64 -- Sec. 2.5: max-margin hyperplane, one-vs-rest
 *                             (each person against all others); solved by dual
 *                             coordinate descent (Hsieh et al., ICML 2008).
 *
 * Parity pins for every function live in tests/test_oracle_*.py. Parity of the
 * neighbour order (which neighbour is p0 and the direction) is NOT fixed by the
 * paper (its figure is lost): it is a convention, checked only for internal
 * consistency (a 90-degree rotation of the crop rotates every code by 2 bits).
 * The SVM trainer's hyper-parameters are likewise a reading, not the paper's;
 * the trainer is pinned against an independent library solver of the same
 * objective.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_MAP_U59 0
#define REF_MAP_FULL256 1
#define REF_MOD_BOTH 0
#define REF_MOD_GREY 1
#define REF_MOD_DEPTH 2

typedef struct {
    const uint8_t *grey;
    const uint16_t *depth;
    int32_t width, height, grey_pitch, depth_pitch; /* pitch in elements */
} lbpf_ref_image;

typedef struct {
    int32_t image, x, y, w, h;
} lbpf_ref_box;

/* ------------------------------------------------------------------------ */
/* Neighbour p of the centre (y, x) is at (y + DY[p], x + DX[p]).            */
/* Order: start at the top-left neighbour and go clockwise (y grows down).   */
static const int DY[8] = {-1, -1, -1, 0, +1, +1, +1, 0};
static const int DX[8] = {-1, 0, +1, +1, +1, 0, -1, -1};

/* Eq. 2: LBP = sum_p s(g_p - g_c) 2^p with s(v) = 1 for v >= 0, else 0.
 * `img` is a row-major plane with `pitch` elements per row; (y, x) must be an
 * interior pixel. */
static int lbp_code_u8(const uint8_t *img, int pitch, int y, int x) {
    int c = img[(size_t)y * pitch + x];
    int code = 0;
    for (int p = 0; p < 8; ++p) {
        int g = img[(size_t)(y + DY[p]) * pitch + (x + DX[p])];
        if (g - c >= 0) code += 1 << p;
    }
    return code;
}

static int lbp_code_u16(const uint16_t *img, int pitch, int y, int x) {
    int c = img[(size_t)y * pitch + x];
    int code = 0;
    for (int p = 0; p < 8; ++p) {
        int g = img[(size_t)(y + DY[p]) * pitch + (x + DX[p])];
        if (g - c >= 0) code += 1 << p;
    }
    return code;
}

/* Exported single-pixel forms, used by the pins. */
int32_t lbpf_ref_lbp_code_u8(const uint8_t *img, int32_t pitch, int32_t y, int32_t x) {
    return lbp_code_u8(img, pitch, y, x);
}
int32_t lbpf_ref_lbp_code_u16(const uint16_t *img, int32_t pitch, int32_t y, int32_t x) {
    return lbp_code_u16(img, pitch, y, x);
}

/* ------------------------------------------------------------------------ */
/* Uniform patterns: count the bit changes while walking once around the
 * eight neighbours (including the wrap from p7 back to p0). */
static int transitions(int code) {
    int t = 0;
    for (int p = 0; p < 8; ++p) {
        int a = (code >> p) & 1;
        int b = (code >> ((p + 1) % 8)) & 1;
        if (a != b) t += 1;
    }
    return t;
}

int32_t lbpf_ref_is_uniform(int32_t code) { return transitions(code) <= 2; }

/* Bin of a code under the uniform-59 mapping: uniform codes get their rank
 * among all uniform codes taken in increasing numeric order (0..57); every
 * other code goes to the last bin, 58. */
int32_t lbpf_ref_uniform_bin(int32_t code) {
    if (!lbpf_ref_is_uniform(code)) return 58;
    int rank = 0;
    for (int c = 0; c < code; ++c)
        if (lbpf_ref_is_uniform(c)) rank += 1;
    return rank;
}

/* Code -> histogram bin for the chosen mapping, tabulated once per call from
 * the definitions above. */
static void build_map(int mapping, uint16_t table[256]) {
    for (int c = 0; c < 256; ++c)
        table[c] = (uint16_t)(mapping == REF_MAP_FULL256 ? c : lbpf_ref_uniform_bin(c));
}

/* ------------------------------------------------------------------------ */
/* Lower median of the non-zero depth values of a w x h crop: sort them and
 * take element (n-1)/2. Returns -1 when the crop has no non-zero value. */
static int cmp_u16(const void *a, const void *b) {
    int x = *(const uint16_t *)a, y = *(const uint16_t *)b;
    return (x > y) - (x < y);
}

int32_t lbpf_ref_median(const uint16_t *depth, int32_t pitch, int32_t w, int32_t h) {
    uint16_t *v = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)w * (size_t)h + 2);
    size_t n = 0;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            uint16_t d = depth[(size_t)y * pitch + x];
            if (d != 0) v[n++] = d;
        }
    int32_t m = -1;
    if (n > 0) {
        qsort(v, n, sizeof(uint16_t), cmp_u16);
        m = v[(n - 1) / 2];
    }
    free(v);
    return m;
}

/* Row band r of `g` bands over a side of length n covers [floor(r*n/g), floor((r+1)*n/g)). */
static int band_start(int r, int n, int g) { return (int)(((int64_t)r * n) / g); }

int32_t lbpf_ref_feature_dim(int32_t grid_x, int32_t grid_y, int32_t mapping, int32_t modality) {
    int nch = modality == REF_MOD_BOTH ? 2 : 1;
    int nb = mapping == REF_MAP_FULL256 ? 256 : 59;
    return nch * grid_x * grid_y * nb;
}

/* In-mask test for a centre depth value: non-zero and |d - m| < window.
 * window <= 0 switches the mask off (every interior pixel counts). */
static int in_mask(int d, int m, int window) {
    if (window <= 0) return 1;
    if (m < 0 || d == 0) return 0;
    return abs(d - m) < window;
}

/* Codes and mask of one crop, for the interior pixels; border entries are 0.
 * Outputs are w*h row-major. */
void lbpf_ref_codes(const uint8_t *grey, int32_t grey_pitch, const uint16_t *depth,
                    int32_t depth_pitch, int32_t w, int32_t h, int32_t window, uint8_t *grey_codes,
                    uint8_t *depth_codes, uint8_t *mask) {
    int m = lbpf_ref_median(depth, depth_pitch, w, h);
    memset(grey_codes, 0, (size_t)w * h);
    memset(depth_codes, 0, (size_t)w * h);
    memset(mask, 0, (size_t)w * h);
    for (int y = 1; y <= h - 2; ++y)
        for (int x = 1; x <= w - 2; ++x) {
            grey_codes[(size_t)y * w + x] = (uint8_t)lbp_code_u8(grey, grey_pitch, y, x);
            depth_codes[(size_t)y * w + x] = (uint8_t)lbp_code_u16(depth, depth_pitch, y, x);
            mask[(size_t)y * w + x] = (uint8_t)in_mask(depth[(size_t)y * depth_pitch + x], m, window);
        }
}

/* Features of one crop: counts (D u32) and L1-normalised feature (D f32).
 * Layout: index = ((channel * grid_y + ry) * grid_x + rx) * nbins + bin, with
 * channel 0 = grey and 1 = depth when both are present. Returns n_in. */
static int64_t one_crop(const uint8_t *G, int gp, const uint16_t *Z, int zp, int w, int h,
                        int grid_x, int grid_y, int mapping, int window, int modality,
                        const uint16_t map[256], uint32_t *counts, float *feat) {
    int nb = mapping == REF_MAP_FULL256 ? 256 : 59;
    int D = lbpf_ref_feature_dim(grid_x, grid_y, mapping, modality);
    int nch = modality == REF_MOD_BOTH ? 2 : 1;
    memset(counts, 0, sizeof(uint32_t) * (size_t)D);
    int m = lbpf_ref_median(Z, zp, w, h);
    int64_t n_in = 0;
    for (int ry = 0; ry < grid_y; ++ry)
        for (int y = band_start(ry, h, grid_y); y < band_start(ry + 1, h, grid_y); ++y) {
            if (y < 1 || y > h - 2) continue;
            for (int rx = 0; rx < grid_x; ++rx)
                for (int x = band_start(rx, w, grid_x); x < band_start(rx + 1, w, grid_x); ++x) {
                    if (x < 1 || x > w - 2) continue;
                    if (!in_mask(Z[(size_t)y * zp + x], m, window)) continue;
                    n_in += 1;
                    int ch = 0;
                    if (modality != REF_MOD_DEPTH) {
                        int b = map[lbp_code_u8(G, gp, y, x)];
                        counts[((size_t)(ch * grid_y + ry) * grid_x + rx) * nb + b] += 1;
                        ch += 1;
                    }
                    if (modality != REF_MOD_GREY) {
                        int b = map[lbp_code_u16(Z, zp, y, x)];
                        counts[((size_t)(ch * grid_y + ry) * grid_x + rx) * nb + b] += 1;
                    }
                }
        }
    /* L1 normalisation: the counts sum to T = channels * n_in. Each entry is
     * the IEEE single-precision quotient count / T (round to nearest even). */
    int64_t T = (int64_t)nch * n_in;
    for (int i = 0; i < D; ++i) {
        if (T == 0) {
            feat[i] = 0.0f;
        } else {
            feat[i] = (float)counts[i] / (float)T;
        }
    }
    return n_in;
}

typedef struct {
    const lbpf_ref_image *imgs;
    const lbpf_ref_box *boxes;
    int32_t n_boxes, grid_x, grid_y, mapping, window, modality;
    const uint16_t *map;
    uint32_t *counts;
    float *feat;
    int64_t *n_in;
    int32_t begin, end;
} feat_job;

static void *feat_worker(void *arg) {
    feat_job *j = (feat_job *)arg;
    int D = lbpf_ref_feature_dim(j->grid_x, j->grid_y, j->mapping, j->modality);
    for (int i = j->begin; i < j->end; ++i) {
        const lbpf_ref_box *b = &j->boxes[i];
        const lbpf_ref_image *im = &j->imgs[b->image];
        const uint8_t *G = im->grey ? im->grey + (size_t)b->y * im->grey_pitch + b->x : NULL;
        const uint16_t *Z = im->depth + (size_t)b->y * im->depth_pitch + b->x;
        int64_t n = one_crop(G, im->grey_pitch, Z, im->depth_pitch, b->w, b->h, j->grid_x,
                             j->grid_y, j->mapping, j->window, j->modality, j->map,
                             j->counts + (size_t)i * D, j->feat + (size_t)i * D);
        if (j->n_in) j->n_in[i] = n;
    }
    return NULL;
}

/* Validate boxes: the image index exists, w,h >= 3, and the box lies inside. */
static int boxes_valid(const lbpf_ref_image *imgs, int32_t n_img, const lbpf_ref_box *boxes,
                       int32_t n_boxes) {
    for (int i = 0; i < n_boxes; ++i) {
        const lbpf_ref_box *b = &boxes[i];
        if (b->image < 0 || b->image >= n_img) return 0;
        const lbpf_ref_image *im = &imgs[b->image];
        if (b->w < 3 || b->h < 3 || b->x < 0 || b->y < 0) return 0;
        if ((int64_t)b->x + b->w > im->width || (int64_t)b->y + b->h > im->height) return 0;
    }
    return 1;
}

/* Features of every box. counts: n_boxes x D (u32), feat: n_boxes x D (f32),
 * n_in: n_boxes (may be NULL). Returns 0, or -1 for invalid arguments. */
int32_t lbpf_ref_features(const lbpf_ref_image *imgs, int32_t n_img, const lbpf_ref_box *boxes,
                          int32_t n_boxes, int32_t grid_x, int32_t grid_y, int32_t mapping,
                          int32_t window, int32_t modality, uint32_t *counts, float *feat,
                          int64_t *n_in, int32_t n_threads) {
    if (grid_x < 1 || grid_y < 1 || (mapping != REF_MAP_U59 && mapping != REF_MAP_FULL256) ||
        modality < 0 || modality > 2 || !boxes_valid(imgs, n_img, boxes, n_boxes))
        return -1;
    uint16_t map[256];
    build_map(mapping, map);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_boxes) n_threads = n_boxes > 0 ? n_boxes : 1;
    feat_job *jobs = (feat_job *)calloc((size_t)n_threads, sizeof(feat_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; ++t) {
        feat_job j = {imgs, boxes, n_boxes, grid_x, grid_y, mapping, window, modality,
                      map, counts, feat, n_in, 0, 0};
        j.begin = (int32_t)(((int64_t)n_boxes * t) / n_threads);
        j.end = (int32_t)(((int64_t)n_boxes * (t + 1)) / n_threads);
        jobs[t] = j;
    }
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, feat_worker, &jobs[t]);
    feat_worker(&jobs[0]);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Warped crops (Sec. 2.1, Eq. 1; Sec. 3 resize). A frame maps crop pixel
 * (x, y) to the source pixel
 *     sx = floor((ux x + vx y + tx) / 65536),  sy = floor((uy x + vy y + ty) / 65536),
 * i.e. p' = x u + y v + t with u = (ux, uy), v = (vx, vy), t = (tx, ty) in
 * 16.16 fixed point, evaluated exactly in 64-bit integers (nearest sample: no
 * interpolation). Every sample must lie inside its plane. */
typedef struct {
    int32_t ux, uy, vx, vy, tx, ty;
} lbpf_ref_frame;

typedef struct {
    int32_t image, w, h;
    lbpf_ref_frame grey, depth;
} lbpf_ref_warp_box;

static int64_t floor_div65536(int64_t a) {
    int64_t q = a / 65536;
    if (a % 65536 != 0 && a < 0) q -= 1; /* C division truncates toward zero */
    return q;
}

/* Sample one plane of element size `esz` through frame f into dst (w*h,
 * pitch w). Returns 0, or -1 if any sample falls outside the plane. */
static int sample_plane(const void *src, int pitch, int width, int height, int esz,
                        const lbpf_ref_frame *f, int w, int h, void *dst) {
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int64_t sx = floor_div65536((int64_t)f->ux * x + (int64_t)f->vx * y + f->tx);
            int64_t sy = floor_div65536((int64_t)f->uy * x + (int64_t)f->vy * y + f->ty);
            if (sx < 0 || sy < 0 || sx >= width || sy >= height) return -1;
            size_t at = (size_t)sy * pitch + (size_t)sx;
            if (esz == 1)
                ((uint8_t *)dst)[(size_t)y * w + x] = ((const uint8_t *)src)[at];
            else
                ((uint16_t *)dst)[(size_t)y * w + x] = ((const uint16_t *)src)[at];
        }
    return 0;
}

/* Features of every warped crop; the same outputs as lbpf_ref_features.
 * Returns 0, or -1 for invalid arguments (image index, side outside
 * 3..1024, a NULL plane the modality needs, a sample outside its plane). */
int32_t lbpf_ref_features_warped(const lbpf_ref_image *imgs, int32_t n_img,
                                 const lbpf_ref_warp_box *boxes, int32_t n_boxes, int32_t grid_x,
                                 int32_t grid_y, int32_t mapping, int32_t window, int32_t modality,
                                 uint32_t *counts, float *feat, int64_t *n_in, int32_t n_threads) {
    if (grid_x < 1 || grid_y < 1 || (mapping != REF_MAP_U59 && mapping != REF_MAP_FULL256) ||
        modality < 0 || modality > 2)
        return -1;
    int D = lbpf_ref_feature_dim(grid_x, grid_y, mapping, modality);
    int use_grey = modality != REF_MOD_DEPTH;
    for (int i = 0; i < n_boxes; ++i) {
        const lbpf_ref_warp_box *b = &boxes[i];
        if (b->image < 0 || b->image >= n_img) return -1;
        if (b->w < 3 || b->h < 3 || b->w > 1024 || b->h > 1024) return -1;
        const lbpf_ref_image *im = &imgs[b->image];
        if (!im->depth || (use_grey && !im->grey)) return -1;
        uint8_t *g = (uint8_t *)malloc((size_t)b->w * b->h);
        uint16_t *z = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)b->w * b->h);
        int bad = sample_plane(im->depth, im->depth_pitch, im->width, im->height, 2, &b->depth,
                               b->w, b->h, z);
        if (use_grey && !bad)
            bad = sample_plane(im->grey, im->grey_pitch, im->width, im->height, 1, &b->grey,
                               b->w, b->h, g);
        if (!use_grey) memset(g, 0, (size_t)b->w * b->h);
        int rc = -1;
        if (!bad) {
            /* The sampled crop is an ordinary image: reuse the plain path. */
            lbpf_ref_image one = {g, z, b->w, b->h, b->w, b->w};
            lbpf_ref_box whole = {0, 0, 0, b->w, b->h};
            int64_t n = 0;
            rc = lbpf_ref_features(&one, 1, &whole, 1, grid_x, grid_y, mapping, window, modality,
                                   counts + (size_t)i * D, feat + (size_t)i * D, &n, 1);
            if (n_in) n_in[i] = n;
        }
        free(g);
        free(z);
        if (rc != 0) return -1;
    }
    (void)n_threads; /* one crop at a time: warped sets in the tests are small */
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Nearest-centre tracking (Sec. 2.3, Fig. 4). Boxes are (x, y, w, h) int32,
 * each with a stream id (only boxes of the same stream are compared). The
 * centre is kept doubled, (2x + w, 2y + h), so it is an exact integer; the
 * distance is the squared Euclidean distance of doubled centres (int64).
 *   match[p] = the current box nearest to track p (lowest index on ties), or
 *              -1 if the stream has none within the gate;
 *   owner[c] = among the tracks whose match is c, the nearest (lowest track
 *              index on ties), or -1: c is a new face.
 * gate2 > 0 limits the distance: a box counts only if the squared distance of
 * the (undoubled) centres is <= gate2, i.e. doubled distance <= 4 gate2. */
void lbpf_ref_track(const int32_t *prev, const int32_t *prev_stream, int32_t P,
                    const int32_t *cur, const int32_t *cur_stream, int32_t C, int64_t gate2,
                    int32_t *match, int32_t *owner) {
    int64_t *best_d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C > 0 ? C : 1));
    for (int c = 0; c < C; ++c) {
        owner[c] = -1;
        best_d[c] = -1;
    }
    for (int p = 0; p < P; ++p) {
        int64_t px = 2 * (int64_t)prev[4 * p] + prev[4 * p + 2];
        int64_t py = 2 * (int64_t)prev[4 * p + 1] + prev[4 * p + 3];
        int best = -1;
        int64_t bd = 0;
        for (int c = 0; c < C; ++c) {
            if (cur_stream[c] != prev_stream[p]) continue;
            int64_t dx = 2 * (int64_t)cur[4 * c] + cur[4 * c + 2] - px;
            int64_t dy = 2 * (int64_t)cur[4 * c + 1] + cur[4 * c + 3] - py;
            int64_t d = dx * dx + dy * dy;
            if (gate2 > 0 && d > 4 * gate2) continue;
            if (best < 0 || d < bd) {
                best = c;
                bd = d;
            }
        }
        match[p] = best;
        if (best >= 0 && (best_d[best] < 0 || bd < best_d[best])) {
            best_d[best] = bd; /* p ascending: an equal distance keeps the lower p */
            owner[best] = p;
        }
    }
    free(best_d);
}

/* ------------------------------------------------------------------------ */
/* Scores: S[n][k] = sum_j W[k][j] * X[n][j] + b[k], in double, j ascending.
 * argmax[n] = the smallest k attaining the largest S[n][k]. Either output may
 * be NULL. */
typedef struct {
    const float *X, *W, *b;
    int64_t N;
    int32_t K, D;
    double *S;
    int32_t *argmax;
    int64_t begin, end;
} score_job;

static void *score_worker(void *arg) {
    score_job *j = (score_job *)arg;
    for (int64_t n = j->begin; n < j->end; ++n) {
        const float *x = j->X + (size_t)n * j->D;
        double best = 0.0;
        int32_t arg_best = -1;
        for (int32_t k = 0; k < j->K; ++k) {
            const float *w = j->W + (size_t)k * j->D;
            double s = 0.0;
            for (int32_t d = 0; d < j->D; ++d) s += (double)w[d] * (double)x[d];
            s += (double)j->b[k];
            if (j->S) j->S[(size_t)n * j->K + k] = s;
            if (arg_best < 0 || s > best) {
                best = s;
                arg_best = k;
            }
        }
        if (j->argmax) j->argmax[n] = arg_best;
    }
    return NULL;
}

void lbpf_ref_score_f64(const float *X, int64_t N, const float *W, const float *b, int32_t K,
                        int32_t D, double *S, int32_t *argmax, int32_t n_threads) {
    if (n_threads < 1) n_threads = 1;
    if (n_threads > N) n_threads = N > 0 ? (int32_t)N : 1;
    score_job *jobs = (score_job *)calloc((size_t)n_threads, sizeof(score_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; ++t) {
        score_job j = {X, W, b, N, K, D, S, argmax, 0, 0};
        j.begin = (N * t) / n_threads;
        j.end = (N * (t + 1)) / n_threads;
        jobs[t] = j;
    }
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, score_worker, &jobs[t]);
    score_worker(&jobs[0]);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
}

/* ------------------------------------------------------------------------ */
/* One-vs-rest linear SVM (L2-regularised hinge loss), trained in double.
 *
 * For class k the labels are y_i = +1 when label_i == k, else -1 (Sec. 2.5:
 * one person is the positive class, every other person the negative one).
 * Each sample is augmented with a constant feature 1 whose weight is the bias,
 * and the features are first multiplied by sigma = 1 / (lower median of the
 * samples' Euclidean norms), so that C = 1 acts on unit-scale data.
 *
 * Problem (primal):  min_w 1/2 |w|^2 + C sum_i max(0, 1 - y_i w.x_i)
 * Dual:              min_a 1/2 a'Qa - sum_i a_i,  0 <= a_i <= C,
 *                    Q_ij = y_i y_j x_i.x_j,  w = sum_i a_i y_i x_i.
 * Dual coordinate descent: visit the coordinates in a seeded random order per
 * epoch; for coordinate i the gradient is G = y_i w.x_i - 1; its projected
 * form PG is G clipped to the feasible directions at the bounds; when PG != 0
 * set a_i <- clip(a_i - G / Q_ii, 0, C) and update w. Stop when the largest
 * |PG| of an epoch falls below eps, or after max_epochs.
 *
 * Outputs W (K x D) and b (K) are in the unscaled feature space:
 * W_k = sigma * w_k[0:D], b_k = w_k[D]. Returns the largest number of epochs
 * any class used.
 */
static uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

typedef struct {
    const double *Xs; /* N x (D+1), scaled and augmented */
    const double *qii;
    const int32_t *labels;
    int32_t N, D1;
    double C, eps;
    int32_t max_epochs;
    uint64_t seed;
    double *Wout, *bout; /* class rows */
    double sigma;
    int32_t D;
    int32_t k_begin, k_end;
    int32_t epochs_used;
} train_job;

static void *train_worker(void *arg) {
    train_job *j = (train_job *)arg;
    int N = j->N, D1 = j->D1;
    double *w = (double *)malloc(sizeof(double) * (size_t)D1);
    double *alpha = (double *)malloc(sizeof(double) * (size_t)N);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int worst = 0;
    for (int k = j->k_begin; k < j->k_end; ++k) {
        memset(w, 0, sizeof(double) * (size_t)D1);
        memset(alpha, 0, sizeof(double) * (size_t)N);
        uint64_t rs = j->seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(k + 1));
        int epoch = 0;
        for (; epoch < j->max_epochs; ++epoch) {
            for (int i = 0; i < N; ++i) perm[i] = i;
            for (int i = N - 1; i > 0; --i) {
                int r = (int)(splitmix64(&rs) % (uint64_t)(i + 1));
                int t = perm[i];
                perm[i] = perm[r];
                perm[r] = t;
            }
            double max_pg = 0.0;
            for (int s = 0; s < N; ++s) {
                int i = perm[s];
                const double *x = j->Xs + (size_t)i * D1;
                double y = j->labels[i] == k ? 1.0 : -1.0;
                double wx = 0.0;
                for (int d = 0; d < D1; ++d) wx += w[d] * x[d];
                double G = y * wx - 1.0;
                double PG = G;
                if (alpha[i] <= 0.0) PG = G < 0.0 ? G : 0.0;
                else if (alpha[i] >= j->C) PG = G > 0.0 ? G : 0.0;
                if (fabs(PG) > max_pg) max_pg = fabs(PG);
                if (PG != 0.0 && j->qii[i] > 0.0) {
                    double a_old = alpha[i];
                    double a_new = a_old - G / j->qii[i];
                    if (a_new < 0.0) a_new = 0.0;
                    if (a_new > j->C) a_new = j->C;
                    alpha[i] = a_new;
                    double step = (a_new - a_old) * y;
                    if (step != 0.0)
                        for (int d = 0; d < D1; ++d) w[d] += step * x[d];
                }
            }
            if (max_pg < j->eps) {
                epoch += 1;
                break;
            }
        }
        if (epoch > worst) worst = epoch;
        for (int d = 0; d < j->D; ++d) j->Wout[(size_t)k * j->D + d] = j->sigma * w[d];
        j->bout[k] = w[j->D];
    }
    j->epochs_used = worst;
    free(w);
    free(alpha);
    free(perm);
    return NULL;
}

int32_t lbpf_ref_train_ovr_f64(const float *X, const int32_t *labels, int32_t N, int32_t D,
                               int32_t K, double C, double eps, int32_t max_epochs, uint64_t seed,
                               double *W, double *b, int32_t n_threads) {
    int D1 = D + 1;
    /* sigma = 1 / lower median of the sample norms (1 if that median is 0). */
    double *norms = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s += (double)X[(size_t)i * D + d] * (double)X[(size_t)i * D + d];
        norms[i] = sqrt(s);
    }
    double sigma = 1.0;
    if (N > 0) {
        qsort(norms, (size_t)N, sizeof(double), cmp_double);
        double med = norms[(N - 1) / 2];
        if (med > 0.0) sigma = 1.0 / med;
    }
    free(norms);
    double *Xs = (double *)malloc(sizeof(double) * (size_t)N * D1);
    double *qii = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int i = 0; i < N; ++i) {
        double q = 0.0;
        for (int d = 0; d < D; ++d) {
            double v = sigma * (double)X[(size_t)i * D + d];
            Xs[(size_t)i * D1 + d] = v;
            q += v * v;
        }
        Xs[(size_t)i * D1 + D] = 1.0;
        qii[i] = q + 1.0;
    }
    if (n_threads < 1) n_threads = 1;
    if (n_threads > K) n_threads = K > 0 ? K : 1;
    train_job *jobs = (train_job *)calloc((size_t)n_threads, sizeof(train_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; ++t) {
        train_job j = {Xs, qii, labels, N, D1, C, eps, max_epochs, seed, W, b, sigma, D, 0, 0, 0};
        j.k_begin = (int32_t)(((int64_t)K * t) / n_threads);
        j.k_end = (int32_t)(((int64_t)K * (t + 1)) / n_threads);
        jobs[t] = j;
    }
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, train_worker, &jobs[t]);
    train_worker(&jobs[0]);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    int worst = 0;
    for (int t = 0; t < n_threads; ++t)
        if (jobs[t].epochs_used > worst) worst = jobs[t].epochs_used;
    free(jobs);
    free(th);
    free(Xs);
    free(qii);
    return worst;
}
