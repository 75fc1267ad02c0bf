/*
 * Sanitizer run of the CPU oracle (test infrastructure, built and run by
 * tests/test_oracle_sanitize.py with AddressSanitizer and
 * UndefinedBehaviorSanitizer). Every exported routine of oracle/lbpf_ref.c runs
 * on seeded synthetic inputs chosen to reach its edges: 3 x 3 crops, crops
 * touching every border of the frame, a whole-frame crop, all-zero depth,
 * constant grey, the 256-bin mapping, single-channel modalities, uneven grids,
 * warped crops whose samples reach the plane's last row and column, tracks with
 * and without a gate, and a small training run. It prints one checksum line and
 * exits 0; any sanitizer report aborts the run with a non-zero status.
 */
#include <stdio.h>

#include "lbpf_ref.c"

/* splitmix64 (Steele, Lea and Flood, OOPSLA 2014). */
static uint64_t sm_state = 0x1504018830000001ull;
static uint64_t sm_next(void) {
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t mix(uint64_t h, uint64_t v) { return (h ^ v) * 0x100000001B3ull; }

int main(void) {
    enum { W0 = 173, H0 = 131, P0 = 181, W1 = 50, H1 = 40 };
    uint8_t *g0 = (uint8_t *)malloc((size_t)P0 * H0);
    uint16_t *z0 = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)P0 * H0);
    uint8_t *g1 = (uint8_t *)malloc((size_t)W1 * H1);
    uint16_t *z1 = (uint16_t *)calloc((size_t)W1 * H1, sizeof(uint16_t)); /* all-zero depth */
    for (int i = 0; i < P0 * H0; ++i) {
        g0[i] = (uint8_t)sm_next();
        const uint64_t r = sm_next();
        z0[i] = (r % 10 == 0) ? 0 : (uint16_t)(500 + (r >> 8) % 3500);
    }
    memset(g1, 77, (size_t)W1 * H1); /* constant grey */
    const lbpf_ref_image imgs[2] = {{g0, z0, W0, H0, P0, P0}, {g1, z1, W1, H1, W1, W1}};
    const lbpf_ref_box boxes[] = {
        {0, 0, 0, 3, 3},      {0, W0 - 3, H0 - 3, 3, 3}, {0, 0, 0, W0, H0},
        {0, 5, 7, 64, 48},    {0, W0 - 70, 0, 70, H0},   {0, 0, H0 - 9, W0, 9},
        {1, 0, 0, W1, H1},    {1, 10, 10, 3, 30},        {0, 100, 20, 73, 111},
    };
    const int nb = (int)(sizeof boxes / sizeof boxes[0]);
    uint64_t h = 0xCBF29CE484222325ull;

    const int grids[3][2] = {{8, 8}, {4, 4}, {3, 5}};
    for (int gi = 0; gi < 3; ++gi)
        for (int mapping = 0; mapping <= 1; ++mapping)
            for (int modality = 0; modality <= 2; ++modality) {
                const int gx = grids[gi][0], gy = grids[gi][1];
                const int D = lbpf_ref_feature_dim(gx, gy, mapping, modality);
                uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nb * D);
                float *feat = (float *)malloc(sizeof(float) * (size_t)nb * D);
                int64_t n_in[16];
                if (lbpf_ref_features(imgs, 2, boxes, nb, gx, gy, mapping, 150, modality, counts,
                                      feat, n_in, 3) != 0)
                    return 2;
                for (size_t i = 0; i < (size_t)nb * D; ++i) h = mix(h, counts[i]);
                for (int i = 0; i < nb; ++i) h = mix(h, (uint64_t)n_in[i]);
                free(counts);
                free(feat);
            }

    /* Invalid boxes are rejected without touching the outputs. */
    const lbpf_ref_box bad = {0, W0 - 2, 0, 3, 3};
    uint32_t c1[2 * 64 * 59];
    float f1[2 * 64 * 59];
    if (lbpf_ref_features(imgs, 2, &bad, 1, 8, 8, REF_MAP_U59, 150, REF_MOD_BOTH, c1, f1, NULL, 1) !=
        -1)
        return 3;

    /* Per-pixel codes and the median of a crop and of an all-zero one. */
    {
        uint8_t gc[64 * 48], zc[64 * 48], mk[64 * 48];
        lbpf_ref_codes(g0 + 7 * P0 + 5, P0, z0 + 7 * P0 + 5, P0, 64, 48, 150, gc, zc, mk);
        for (int i = 0; i < 64 * 48; ++i) h = mix(h, (uint64_t)gc[i] | (uint64_t)zc[i] << 8 | (uint64_t)mk[i] << 16);
        h = mix(h, (uint64_t)(int64_t)lbpf_ref_median(z1, W1, W1, H1));
        h = mix(h, (uint64_t)(int64_t)lbpf_ref_median(z0, P0, W0, H0));
    }

    /* Warped crops: identity frames, a 2x downscale reaching the last
     * row and column, and a frame that leaves the plane (rejected). */
    {
        const int D = lbpf_ref_feature_dim(8, 8, REF_MAP_U59, REF_MOD_BOTH);
        lbpf_ref_warp_box wb[3];
        memset(wb, 0, sizeof wb);
        wb[0].image = 0; wb[0].w = 20; wb[0].h = 20;
        wb[0].grey = (lbpf_ref_frame){65536, 0, 0, 65536, 3 * 65536, 4 * 65536};
        wb[0].depth = wb[0].grey;
        wb[1].image = 0; wb[1].w = (W0 + 1) / 2; wb[1].h = (H0 + 1) / 2;
        wb[1].grey = (lbpf_ref_frame){2 * 65536, 0, 0, 2 * 65536, 0, 0};
        wb[1].depth = wb[1].grey;
        wb[2] = wb[1];
        wb[2].w = wb[1].w + 1;
        uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)D);
        float *feat = (float *)malloc(sizeof(float) * 3 * (size_t)D);
        int64_t n_in[3];
        if (lbpf_ref_features_warped(imgs, 2, wb, 2, 8, 8, REF_MAP_U59, 150, REF_MOD_BOTH, counts,
                                     feat, n_in, 1) != 0)
            return 4;
        for (size_t i = 0; i < 2 * (size_t)D; ++i) h = mix(h, counts[i]);
        if (lbpf_ref_features_warped(imgs, 2, wb + 2, 1, 8, 8, REF_MAP_U59, 150, REF_MOD_BOTH,
                                     counts, feat, n_in, 1) != -1)
            return 5;
        free(counts);
        free(feat);
    }

    /* Scores and argmax over the feature rows of the boxes. */
    {
        const int D = lbpf_ref_feature_dim(8, 8, REF_MAP_U59, REF_MOD_BOTH), K = 7;
        uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nb * D);
        float *X = (float *)malloc(sizeof(float) * (size_t)nb * D);
        float *Wt = (float *)malloc(sizeof(float) * (size_t)K * D);
        float b[7];
        double S[16 * 7];
        int32_t am[16];
        if (lbpf_ref_features(imgs, 2, boxes, nb, 8, 8, REF_MAP_U59, 150, REF_MOD_BOTH, counts, X,
                              NULL, 2) != 0)
            return 6;
        for (int i = 0; i < K * D; ++i) Wt[i] = (float)((int64_t)(sm_next() % 2001) - 1000) / 1000.0f;
        for (int k = 0; k < K; ++k) b[k] = (float)k * 0.01f;
        lbpf_ref_score_f64(X, nb, Wt, b, K, D, S, am, 3);
        for (int i = 0; i < nb; ++i) h = mix(h, (uint64_t)am[i]);
        free(counts);
        free(X);
        free(Wt);
    }

    /* A small one-vs-rest training run. */
    {
        enum { N = 30, D = 16, K = 3 };
        float X[N * D];
        int32_t labels[N];
        double Wd[K * (D + 1)], bd[K];
        for (int i = 0; i < N; ++i) {
            labels[i] = i % K;
            for (int d = 0; d < D; ++d)
                X[i * D + d] = (float)((sm_next() % 1000) / 1000.0) + (d % K == labels[i] ? 1.0f : 0.0f);
        }
        if (lbpf_ref_train_ovr_f64(X, labels, N, D, K, 1.0, 1e-6, 200, 7, Wd, bd, 2) < 0) return 7;
        for (int k = 0; k < K; ++k) h = mix(h, (uint64_t)(bd[k] > 0));
    }

    /* Tracking with and without a gate, an empty stream and no tracks. */
    {
        const int32_t prev[] = {10, 10, 40, 40, 100, 50, 30, 30, 5, 5, 20, 20};
        const int32_t prev_stream[] = {0, 0, 1};
        const int32_t cur[] = {12, 11, 40, 40, 300, 300, 10, 10, 90, 52, 30, 30};
        const int32_t cur_stream[] = {0, 2, 0};
        int32_t match[3], owner[3];
        lbpf_ref_track(prev, prev_stream, 3, cur, cur_stream, 3, 0, match, owner);
        for (int i = 0; i < 3; ++i) h = mix(h, (uint64_t)(match[i] + 2) << 8 | (uint64_t)(owner[i] + 2));
        lbpf_ref_track(prev, prev_stream, 3, cur, cur_stream, 3, 100, match, owner);
        for (int i = 0; i < 3; ++i) h = mix(h, (uint64_t)(match[i] + 2) << 8 | (uint64_t)(owner[i] + 2));
        lbpf_ref_track(prev, prev_stream, 0, cur, cur_stream, 3, 0, match, owner);
        for (int i = 0; i < 3; ++i) h = mix(h, (uint64_t)(owner[i] + 2));
    }

    free(g0);
    free(z0);
    free(g1);
    free(z1);
    printf("oracle sanitize ok %016llx\n", (unsigned long long)h);
    return 0;
}
