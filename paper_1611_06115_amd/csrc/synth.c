/*
 * synth.c -- seeded synthetic DNA text generators (ASCII output).
 *
 * Input generation only: this file holds none of the scan's arithmetic (no
 * codes, masks or counts).  It writes the letters A, C, G, T and is shared by
 * the tests, the benchmark and the oracle's inputs.
 *
 * Randomness is counter based: draw(key, i) = mix64(key + G * (i + 1)) with
 * G = 0x9E3779B97F4A7C15 and mix64 the SplitMix64 output function (Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014).  Any block of the text can therefore be regenerated independently,
 * which is what lets threads split the work.  Each 64-bit draw supplies four
 * 16-bit uniforms; a base is chosen by comparing its uniform with 16-bit
 * cumulative thresholds.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + GOLDEN * (i + 1)); }

uint64_t pms_key(uint64_t seed, uint64_t stream) { return mix64(seed * GOLDEN + stream + 1); }

uint64_t pms_draw(uint64_t key, uint64_t i) { return draw(key, i); }

static const char LETTER[4] = {'A', 'C', 'G', 'T'};

static inline int pick(uint32_t u16, const uint16_t* thr /* 3 cumulative thresholds */) {
    return (u16 >= thr[0]) + (u16 >= thr[1]) + (u16 >= thr[2]);
}

typedef struct {
    uint8_t* out;
    uint64_t n, key, lo, hi; /* draw indices [lo, hi) (iid) or chunks (markov) */
    const uint16_t* thr;
    const uint16_t* start;
    uint64_t chunk;
} job_t;

static void* iid_worker(void* a) {
    job_t* j = (job_t*)a;
    for (uint64_t d = j->lo; d < j->hi; ++d) {
        uint64_t r = draw(j->key, d);
        for (int q = 0; q < 4; ++q) {
            uint64_t i = 4 * d + (uint64_t)q;
            if (i >= j->n) break;
            j->out[i] = (uint8_t)LETTER[pick((uint32_t)(r >> (16 * q)) & 0xFFFFu, j->thr)];
        }
    }
    return NULL;
}

static int run_jobs(job_t* jobs, int threads, void* (*fn)(void*)) {
    pthread_t* tid = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    if (!tid) return -1;
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, fn, &jobs[t]) != 0) break;
        started = t;
    }
    fn(&jobs[0]);
    for (int t = started + 1; t < threads; ++t) fn(&jobs[t]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    free(tid);
    return 0;
}

/* i.i.d. bases with cumulative 16-bit thresholds thr[0..2] (P(A), P(A+C),
 * P(A+C+G) times 65536). */
int pms_iid(uint8_t* out, uint64_t n, uint64_t key, const uint16_t* thr, int threads) {
    if (threads < 1) threads = 1;
    uint64_t draws = (n + 3) / 4;
    job_t* jobs = (job_t*)calloc((size_t)threads, sizeof(job_t));
    if (!jobs) return -1;
    for (int t = 0; t < threads; ++t) {
        jobs[t].out = out;
        jobs[t].n = n;
        jobs[t].key = key;
        jobs[t].thr = thr;
        jobs[t].lo = draws * (uint64_t)t / (uint64_t)threads;
        jobs[t].hi = draws * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    int rc = run_jobs(jobs, threads, iid_worker);
    free(jobs);
    return rc;
}

static void* markov_worker(void* a) {
    job_t* j = (job_t*)a;
    for (uint64_t c = j->lo; c < j->hi; ++c) {
        uint64_t base = c * j->chunk;
        uint64_t len = j->n - base < j->chunk ? j->n - base : j->chunk;
        uint64_t ckey = mix64(j->key ^ (GOLDEN * (c + 1)));
        /* start context from the stationary law: 63 cumulative thresholds */
        uint32_t u = (uint32_t)(draw(ckey, 0) & 0xFFFFu);
        unsigned ctx = 0;
        while (ctx < 63 && u >= j->start[ctx]) ++ctx;
        uint64_t r = 0;
        for (uint64_t s = 0; s < len; ++s) {
            if ((s & 3) == 0) r = draw(ckey, 1 + s / 4);
            uint32_t v = (uint32_t)(r >> (16 * (s & 3))) & 0xFFFFu;
            int b = pick(v, j->thr + 3 * ctx);
            j->out[base + s] = (uint8_t)LETTER[b];
            ctx = ((ctx << 2) | (unsigned)b) & 63u;
        }
    }
    return NULL;
}

/* Order-3 Markov chain.  thr holds 64 rows of 3 cumulative 16-bit thresholds,
 * row index = (b[-3] << 4) | (b[-2] << 2) | b[-1] with bases indexed A,C,G,T;
 * start holds 63 cumulative thresholds of the stationary context law.  The
 * text is generated in independent chunks of `chunk` bases, each starting
 * from a context drawn from that law. */
int pms_markov3(uint8_t* out, uint64_t n, uint64_t key, const uint16_t* thr,
                const uint16_t* start, uint64_t chunk, int threads) {
    if (threads < 1) threads = 1;
    if (chunk == 0) return -1;
    uint64_t nchunks = (n + chunk - 1) / chunk;
    job_t* jobs = (job_t*)calloc((size_t)threads, sizeof(job_t));
    if (!jobs) return -1;
    for (int t = 0; t < threads; ++t) {
        jobs[t].out = out;
        jobs[t].n = n;
        jobs[t].key = key;
        jobs[t].thr = thr;
        jobs[t].start = start;
        jobs[t].chunk = chunk;
        jobs[t].lo = nchunks * (uint64_t)t / (uint64_t)threads;
        jobs[t].hi = nchunks * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    int rc = run_jobs(jobs, threads, markov_worker);
    free(jobs);
    return rc;
}
