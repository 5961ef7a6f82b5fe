/*
 * oracle.c -- CPU oracle for the k-mismatch character-class scan.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously correct brute
 * force of what the scan computes.  Only the tests, the smoke check and the
 * benchmark's cpu_baseline leg load it; the product path never does.  It
 * shares no code, header or table with the HIP library: class membership
 * comes from the IUPAC meanings written out below, not from any code table,
 * prime product or pair dictionary.
 *
 * What it computes (0-based positions):
 *   pattern p = (S_0 .. S_{m-1}), each S_j a subset of {A,C,G,T}
 *   c_i = #{ j in [0,m) : t[i+j] not in S_j },   i = 0 .. n-m
 *   result = [(i, c_i) for ascending i with c_i <= k]
 * The class-match rule and the "at most k mismatches" rule are the paper's
 * problem statement (Sect. 1.1); eq. (4) of Sect. 2.4 sums exactly these
 * per-position mismatch indicators.  A window is abandoned as soon as its
 * count exceeds k (the early stop of Sect. 2.4; Table 4 abandons window 2 of
 * the worked example at its third mismatch with k = 2).  Abandoning never
 * changes the result: it only skips windows that are already rejected.
 *
 * Threads follow Sect. 2.6: the windows are cut into T contiguous ranges,
 * each scanned by its own thread reading m-1 bases past its last window
 * start; the per-range hit lists are concatenated in range order.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PMO_OK 0
#define PMO_ERR_ARG (-1)
#define PMO_ERR_SYMBOL (-2)
#define PMO_ERR_NOMEM (-3)

/* Bases are named by index 0..3 in alphabetical order A, C, G, T.  A class
 * is the set of member bases, held as a 4-bit set (bit b <=> base b). */
static int base_of(uint8_t ch) {
    switch (ch) {
        case 'A': case 'a': return 0;
        case 'C': case 'c': return 1;
        case 'G': case 'g': return 2;
        case 'T': case 't': return 3;
        default: return -1;
    }
}

static unsigned set_of_names(const char* names) {
    unsigned s = 0;
    for (; *names; ++names) s |= 1u << base_of((uint8_t)*names);
    return s;
}

/* IUPAC one-letter classes, the first column of Table 2 (Sect. 2.2).  '-'
 * marks a missing or erroneous pattern symbol; it matches no base. */
static int iupac_set(uint8_t ch, unsigned* out) {
    const char* names;
    switch (ch) {
        case 'A': case 'a': names = "A"; break;
        case 'C': case 'c': names = "C"; break;
        case 'G': case 'g': names = "G"; break;
        case 'T': case 't': names = "T"; break;
        case 'M': case 'm': names = "AC"; break;
        case 'R': case 'r': names = "AG"; break;
        case 'W': case 'w': names = "AT"; break;
        case 'S': case 's': names = "CG"; break;
        case 'Y': case 'y': names = "CT"; break;
        case 'K': case 'k': names = "GT"; break;
        case 'V': case 'v': names = "ACG"; break;
        case 'H': case 'h': names = "ACT"; break;
        case 'D': case 'd': names = "AGT"; break;
        case 'B': case 'b': names = "CGT"; break;
        case 'N': case 'n': names = "ACGT"; break;
        case '-': names = ""; break;
        default: return 0;
    }
    *out = set_of_names(names);
    return 1;
}

/* Parse a pattern: IUPAC letters, '-', and bracketed classes such as
 * "[CGT]" (the notation of the examples in Sect. 1.1 and 2.5), whose set is
 * the union of the letters inside.  Writes one 4-bit set per position.
 * Returns the pattern length, or a negative error code. */
int64_t pmo_parse(const char* pat, uint64_t len, uint8_t* sets, uint64_t cap) {
    uint64_t m = 0;
    for (uint64_t i = 0; i < len; ++i) {
        unsigned s = 0;
        if (pat[i] == '[') {
            uint64_t j = i + 1;
            int any = 0;
            while (j < len && pat[j] != ']') {
                unsigned t;
                if (pat[j] == '-' || pat[j] == '[' || !iupac_set((uint8_t)pat[j], &t))
                    return PMO_ERR_SYMBOL;
                s |= t;
                any = 1;
                ++j;
            }
            if (j >= len || !any) return PMO_ERR_SYMBOL;
            i = j;
        } else if (!iupac_set((uint8_t)pat[i], &s)) {
            return PMO_ERR_SYMBOL;
        }
        if (m < cap) sets[m] = (uint8_t)s;
        ++m;
    }
    return (int64_t)m;
}

/* Index of the first byte that is not A, C, G or T (either case), or -1. */
int64_t pmo_first_bad(const uint8_t* text, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i)
        if (base_of(text[i]) < 0) return (int64_t)i;
    return -1;
}

/* Full mismatch count of every window, no early stop (for small inputs). */
int pmo_counts(const uint8_t* text, uint64_t n, const uint8_t* sets, uint64_t m,
               uint32_t* counts) {
    if (m == 0) return PMO_ERR_ARG;
    if (pmo_first_bad(text, n) >= 0) return PMO_ERR_SYMBOL;
    if (m > n) return PMO_OK;
    for (uint64_t i = 0; i + m <= n; ++i) {
        uint32_t c = 0;
        for (uint64_t j = 0; j < m; ++j)
            if (!((sets[j] >> base_of(text[i + j])) & 1u)) ++c;
        counts[i] = c;
    }
    return PMO_OK;
}

typedef struct {
    const uint8_t* text;
    const uint8_t* sets;
    uint64_t m, k, first, last; /* windows [first, last) */
    int64_t* pos;
    uint16_t* cnt;
    uint64_t len, cap;
    int err;
} range_job;

static void push_hit(range_job* r, uint64_t i, uint64_t c) {
    if (r->err) return;
    if (r->len == r->cap) {
        uint64_t nc = r->cap ? 2 * r->cap : 1024;
        int64_t* np = (int64_t*)realloc(r->pos, nc * sizeof(int64_t));
        if (!np) { r->err = PMO_ERR_NOMEM; return; }
        r->pos = np;
        uint16_t* nq = (uint16_t*)realloc(r->cnt, nc * sizeof(uint16_t));
        if (!nq) { r->err = PMO_ERR_NOMEM; return; }
        r->cnt = nq;
        r->cap = nc;
    }
    r->pos[r->len] = (int64_t)i;
    r->cnt[r->len] = (uint16_t)c;
    r->len++;
}

static void* scan_range(void* arg) {
    range_job* r = (range_job*)arg;
    for (uint64_t i = r->first; i < r->last; ++i) {
        uint64_t c = 0;
        uint64_t j = 0;
        for (; j < r->m; ++j) {
            if (!((r->sets[j] >> base_of(r->text[i + j])) & 1u)) {
                ++c;
                if (c > r->k) break; /* early stop: the window is rejected */
            }
        }
        if (c <= r->k) push_hit(r, i, c);
    }
    return NULL;
}

/* Scan windows [win_begin, win_end) (clipped to [0, n-m+1)) with T threads.
 * Writes the first `cap` hits in ascending position order and returns the
 * total number of hits, or a negative error code.  k above 65535 is
 * rejected because counts are reported as 16-bit values. */
int64_t pmo_scan_range(const uint8_t* text, uint64_t n, const uint8_t* sets, uint64_t m,
                       uint64_t k, uint64_t win_begin, uint64_t win_end, int threads,
                       int64_t* pos, uint16_t* cnt, uint64_t cap) {
    if (m == 0 || k > 65535 || threads < 1) return PMO_ERR_ARG;
    if (pmo_first_bad(text, n) >= 0) return PMO_ERR_SYMBOL;
    if (m > n) return 0;
    uint64_t nw = n - m + 1;
    if (win_end > nw) win_end = nw;
    if (win_begin >= win_end) return 0;
    uint64_t span = win_end - win_begin;
    if ((uint64_t)threads > span) threads = (int)span;
    range_job* jobs = (range_job*)calloc((size_t)threads, sizeof(range_job));
    pthread_t* tid = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return PMO_ERR_NOMEM; }
    for (int t = 0; t < threads; ++t) {
        jobs[t].text = text;
        jobs[t].sets = sets;
        jobs[t].m = m;
        jobs[t].k = k;
        jobs[t].first = win_begin + span * (uint64_t)t / (uint64_t)threads;
        jobs[t].last = win_begin + span * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, scan_range, &jobs[t]) != 0) break;
        started = t;
    }
    scan_range(&jobs[0]);
    for (int t = started + 1; t < threads; ++t) scan_range(&jobs[t]); /* not started */
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    int64_t total = 0;
    int err = 0;
    for (int t = 0; t < threads; ++t) {
        if (jobs[t].err) err = jobs[t].err;
        for (uint64_t h = 0; h < jobs[t].len; ++h) {
            if ((uint64_t)total < cap) {
                pos[total] = jobs[t].pos[h];
                cnt[total] = jobs[t].cnt[h];
            }
            ++total;
        }
        free(jobs[t].pos);
        free(jobs[t].cnt);
    }
    free(jobs);
    free(tid);
    return err ? err : total;
}

int64_t pmo_scan(const uint8_t* text, uint64_t n, const uint8_t* sets, uint64_t m, uint64_t k,
                 int threads, int64_t* pos, uint16_t* cnt, uint64_t cap) {
    return pmo_scan_range(text, n, sets, m, k, 0, UINT64_MAX, threads, pos, cnt, cap);
}
