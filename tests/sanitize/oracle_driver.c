/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (oracle.c, included here as one translation unit, built without
 * OpenMP): every filter, window and evaluator kind on small 8- and 16-bit
 * images (1 x 1 and ragged shapes, zero pixels, uniform patches), whole
 * images, pixel lists and per-pixel inspection. Exits 0 when nothing
 * aborted. Built and run by tests/test_sanitizers.py. */
#include "../../oracle/oracle.c"

#include <stdio.h>

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next_u64(void) {   /* xorshift64 */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static void fill(void* img, int h, int w, int bpc, int mode) {
    for (int i = 0; i < h * w * 3; ++i) {
        uint32_t v = (uint32_t)(next_u64() % (bpc == 1 ? 256u : 65536u));
        if (mode == 1 && (i / 3) % 5 == 0) v = 0;        /* zero pixels */
        if (mode == 2) v = bpc == 1 ? 77u : 19789u;      /* uniform */
        if (bpc == 1) ((uint8_t*)img)[i] = (uint8_t)v;
        else ((uint16_t*)img)[i] = (uint16_t)v;
    }
}

int main(void) {
    static const int shapes[][2] = {{1, 1}, {1, 6}, {7, 1}, {5, 3}, {9, 11}};
    orc_cfg_t cfg;
    long runs = 0;
    for (int filter = 0; filter <= 4; ++filter)
        for (int window = 3; window <= 7; window += 2)
            for (int kind = 0; kind <= 3; ++kind)
                for (int bpc = 1; bpc <= 2; ++bpc)
                    for (int s = 0; s < 5; ++s)
                        for (int mode = 0; mode < 3; ++mode) {
                            memset(&cfg, 0, sizeof cfg);
                            cfg.filter = filter;
                            cfg.window = window;
                            cfg.param = filter == 1 ? 0.25 : 0.33;
                            cfg.acos_ap.kind = kind;
                            cfg.acos_ap.n_lo = cfg.acos_ap.n_hi = 4;
                            for (int k = 0; k < 4; ++k) {
                                cfg.acos_ap.lo[k] = 1.0 / (k + 1);
                                cfg.acos_ap.hi[k] = 0.5 / (k + 1);
                            }
                            cfg.exp_ap.kind = kind % 3;
                            cfg.exp_ap.n = 5;
                            cfg.exp_ap.n_q = 5;
                            cfg.exp_ap.cutoff = 10.0;
                            for (int k = 0; k < 5; ++k) {
                                cfg.exp_ap.c[k] = k % 2 ? -1.0 / (k + 1) : 1.0 / (k + 1);
                                cfg.exp_ap.q[k] = 1.0 / (k + 1);
                            }
                            cfg.ent_ap.kind = kind % 3;
                            cfg.ent_ap.n_p = cfg.ent_ap.n_q = 5;
                            cfg.ent_ap.cutoff = kind == 1 ? 0.05 : (kind == 3 ? 0.2 : 0.0);
                            for (int k = 0; k < 5; ++k) {
                                cfg.ent_ap.p[k] = 0.1 * (k + 1);
                                cfg.ent_ap.q[k] = 1.0 + k;
                            }
                            const int h = shapes[s][0], w = shapes[s][1];
                            const size_t bytes = (size_t)h * w * 3 * bpc;
                            void* src = malloc(bytes);
                            void* dst = malloc(bytes);
                            fill(src, h, w, bpc, mode);
                            const int64_t pitch = (int64_t)w * 3;   /* in channels */
                            orc_filter(src, h, w, bpc, pitch, dst, pitch, &cfg, NULL, NULL, 0, 1);
                            int32_t ys[3] = {0, h - 1, h / 2}, xs[3] = {w - 1, 0, w / 2};
                            orc_filter(src, h, w, bpc, pitch, dst, pitch, &cfg, ys, xs, 3, 1);
                            double out[4 + 3 * ORC_MAXN];
                            (void)orc_inspect(src, h, w, bpc, pitch, &cfg, h / 2, w / 2, out);
                            free(src);
                            free(dst);
                            ++runs;
                        }
    printf("oracle: %ld configurations\n", runs);
    return 0;
}
