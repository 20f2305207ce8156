/*
 * Plain C transcription of the integer-mode oracle (oracle/model.py).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests and by the CPU baseline leg of
 * the benchmark, never by the product library.  Shares no code with it.
 *
 * The simulator follows Section 4.1 step by step: one FIFO software queue per
 * engine filled in launch order, ready heads started, end times estimated,
 * time advanced to the earliest end.  Concurrent HtD and DtH transfers advance
 * at p_htd/q and p_dth/q of their solo speed (the reading of Section 4.2.1 used
 * throughout); remaining transfer work is exact in 1/q solo-ns units and every
 * completion estimate is rounded up to a whole nanosecond.
 *
 * Orderings are enumerated in lexicographic order (rank 0 = identity) with the
 * textbook successor step; a worker thread that starts inside the range decodes
 * its first ordering from the factorial-base digits of its starting rank.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OMAXN 16
enum { K_HTD = 0, K_KER = 1, K_DTH = 2 };

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/* events (optional): ev[task*6 + kind*2 + {0,1}] = start, end */
int64_t oracle_simulate(const int64_t *tasks, int n, const int *order, int q, int p_htd,
                        int p_dth, int dma, int64_t *ev) {
    int neng = dma == 2 ? 3 : 2;
    int qkind[3][2 * OMAXN], qtask[3][2 * OMAXN], qlen[3] = {0, 0, 0}, qhead[3] = {0, 0, 0};
    int run_kind[3] = {-1, -1, -1}, run_task[3] = {-1, -1, -1};
    int64_t left[3] = {0, 0, 0}, rate[3], est[3];
    unsigned char done[3][OMAXN];
    memset(done, 0, sizeof(done));
    for (int j = 0; j < n; ++j) {
        if (dma == 2) {
            qkind[0][qlen[0]] = K_HTD; qtask[0][qlen[0]++] = order[j];
            qkind[1][qlen[1]] = K_KER; qtask[1][qlen[1]++] = order[j];
            qkind[2][qlen[2]] = K_DTH; qtask[2][qlen[2]++] = order[j];
        } else {
            qkind[0][qlen[0]] = K_HTD; qtask[0][qlen[0]++] = order[j];
            qkind[1][qlen[1]] = K_KER; qtask[1][qlen[1]++] = order[j];
        }
    }
    if (dma == 1)
        for (int j = 0; j < n; ++j) { qkind[0][qlen[0]] = K_DTH; qtask[0][qlen[0]++] = order[j]; }

    int64_t t = 0, total = 0;
    for (;;) {
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 && left[e] == 0) {
                    done[run_kind[e]][run_task[e]] = 1;
                    if (ev) ev[run_task[e] * 6 + run_kind[e] * 2 + 1] = t;
                    if (t > total) total = t;
                    run_kind[e] = -1;
                    changed = 1;
                }
            }
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] < 0 && qhead[e] < qlen[e]) {
                    int kind = qkind[e][qhead[e]], x = qtask[e][qhead[e]];
                    int ready = kind == K_HTD ? 1 : (kind == K_KER ? done[K_HTD][x] : done[K_KER][x]);
                    if (ready) {
                        qhead[e]++;
                        run_kind[e] = kind;
                        run_task[e] = x;
                        left[e] = tasks[x * 3 + kind] * (kind == K_KER ? 1 : q);
                        if (ev) ev[x * 6 + kind * 2] = t;
                        changed = 1;
                    }
                }
            }
        }
        int busy = 0, any_h = 0, any_d = 0;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] >= 0) {
                busy = 1;
                if (run_kind[e] == K_HTD) any_h = 1;
                if (run_kind[e] == K_DTH) any_d = 1;
            }
        }
        if (!busy) break;
        int overlap = any_h && any_d;
        int64_t delta = INT64_MAX;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            if (run_kind[e] == K_KER) rate[e] = 1;
            else if (overlap) rate[e] = run_kind[e] == K_HTD ? p_htd : p_dth;
            else rate[e] = q;
            est[e] = ceil_div(left[e], rate[e]);
            if (est[e] < delta) delta = est[e];
        }
        t += delta;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            if (est[e] == delta) left[e] = 0;
            else left[e] -= rate[e] * delta;
        }
    }
    return total;
}

/* ---------------------------------------------------------------- enumeration */

static void decode_rank(int n, uint64_t r, int *perm) {
    int rest[OMAXN];
    uint64_t fact[OMAXN + 1];
    fact[0] = 1;
    for (int i = 1; i <= n; ++i) fact[i] = fact[i - 1] * (uint64_t)i;
    for (int i = 0; i < n; ++i) rest[i] = i;
    int m = n;
    for (int i = 0; i < n; ++i) {
        uint64_t block = fact[n - 1 - i];
        int c = (int)(r / block);
        r %= block;
        perm[i] = rest[c];
        for (int j = c; j < m - 1; ++j) rest[j] = rest[j + 1];
        --m;
    }
}

/* lexicographic successor; returns 0 after the last ordering */
static int next_perm(int n, int *a) {
    int i = n - 2;
    while (i >= 0 && a[i] > a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] < a[i]) --j;
    int tmp = a[i]; a[i] = a[j]; a[j] = tmp;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) { tmp = a[l]; a[l] = a[r]; a[r] = tmp; }
    return 1;
}

typedef struct {
    int64_t min_ns, max_ns;
    uint64_t argmin, argmax;
    uint64_t sum_lo, sum_hi, count, fingerprint;
} oracle_summary;

typedef struct {
    const int64_t *tasks;
    int n, q, p_htd, p_dth, dma;
    uint64_t lo, hi, stride;
    int64_t *per_order; /* indexed by rank - base, may be NULL */
    uint64_t base;
    oracle_summary s;
    unsigned __int128 sum;
} job_t;

static void *worker(void *arg) {
    job_t *j = (job_t *)arg;
    int perm[OMAXN];
    j->s.min_ns = INT64_MAX; j->s.max_ns = -1; j->s.argmin = 0; j->s.argmax = 0;
    j->s.count = 0; j->s.fingerprint = 0; j->sum = 0;
    if (j->lo >= j->hi) return NULL;
    if (j->stride <= 1) {
        decode_rank(j->n, j->lo, perm);
        for (uint64_t r = j->lo; r < j->hi; ++r) {
            int64_t T = oracle_simulate(j->tasks, j->n, perm, j->q, j->p_htd, j->p_dth, j->dma, NULL);
            if (T < j->s.min_ns) { j->s.min_ns = T; j->s.argmin = r; }
            if (T > j->s.max_ns) { j->s.max_ns = T; j->s.argmax = r; }
            j->sum += (unsigned __int128)T;
            j->s.fingerprint += (2 * r + 1) * (uint64_t)T;
            j->s.count++;
            if (j->per_order) j->per_order[r - j->base] = T;
            next_perm(j->n, perm);
        }
    } else {
        for (uint64_t r = j->lo; r < j->hi; r += j->stride) {
            decode_rank(j->n, r, perm);
            int64_t T = oracle_simulate(j->tasks, j->n, perm, j->q, j->p_htd, j->p_dth, j->dma, NULL);
            if (T < j->s.min_ns) { j->s.min_ns = T; j->s.argmin = r; }
            if (T > j->s.max_ns) { j->s.max_ns = T; j->s.argmax = r; }
            j->sum += (unsigned __int128)T;
            j->s.fingerprint += (2 * r + 1) * (uint64_t)T;
            j->s.count++;
        }
    }
    return NULL;
}

/*
 * Evaluate the orderings with rank in [lo, hi) (every stride-th one when
 * stride > 1) on nthreads threads.  per_order (optional, contiguous ranks
 * only) receives T at index rank - lo.
 */
int oracle_exhaustive(const int64_t *tasks, int n, int q, int p_htd, int p_dth, int dma,
                      uint64_t lo, uint64_t hi, uint64_t stride, int nthreads,
                      int64_t *per_order, oracle_summary *out) {
    if (n < 1 || n > OMAXN || nthreads < 1 || hi < lo) return -1;
    if (stride < 1) stride = 1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t steps = (hi - lo + stride - 1) / stride;
    uint64_t per = (steps + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int i = 0; i < nthreads; ++i) {
        job_t *j = &jobs[i];
        j->tasks = tasks; j->n = n; j->q = q; j->p_htd = p_htd; j->p_dth = p_dth; j->dma = dma;
        uint64_t a = (uint64_t)i * per, b = a + per;
        if (a > steps) a = steps;
        if (b > steps) b = steps;
        j->lo = lo + a * stride;
        j->hi = lo + b * stride;
        if (j->hi > hi) j->hi = hi;
        j->stride = stride;
        j->per_order = stride == 1 ? per_order : NULL;
        j->base = lo;
        pthread_create(&th[i], NULL, worker, j);
    }
    oracle_summary s;
    s.min_ns = INT64_MAX; s.max_ns = -1; s.argmin = 0; s.argmax = 0; s.count = 0; s.fingerprint = 0;
    unsigned __int128 sum = 0;
    for (int i = 0; i < nthreads; ++i) {
        pthread_join(th[i], NULL);
        job_t *j = &jobs[i];
        if (j->s.count == 0) continue;
        /* threads hold increasing rank ranges: strict comparisons keep the lowest rank */
        if (j->s.min_ns < s.min_ns) { s.min_ns = j->s.min_ns; s.argmin = j->s.argmin; }
        if (j->s.max_ns > s.max_ns) { s.max_ns = j->s.max_ns; s.argmax = j->s.argmax; }
        sum += j->sum;
        s.fingerprint += j->s.fingerprint;
        s.count += j->s.count;
    }
    s.sum_lo = (uint64_t)sum;
    s.sum_hi = (uint64_t)(sum >> 64);
    *out = s;
    free(jobs);
    free(th);
    return 0;
}

/* T for m given orderings (orders is m x n bytes, row-major). */
int oracle_eval_orders(const int64_t *tasks, int n, int q, int p_htd, int p_dth, int dma,
                       const uint8_t *orders, int64_t m, int64_t *out) {
    if (n < 1 || n > OMAXN) return -1;
    int perm[OMAXN];
    for (int64_t i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) perm[j] = orders[i * n + j];
        out[i] = oracle_simulate(tasks, n, perm, q, p_htd, p_dth, dma, NULL);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Workers with dependent tasks (oracle/rounds.py, NoReorder setup): task
 * (w, r) at index w * R + r; seq holds the T * R task indices in launch order,
 * round by round.  The HtD of (w, r) is ready once the DtH of (w, r - 1) has
 * ended.  Two DMA engines: three FIFO queues in seq order.  One DMA engine:
 * the transfer queue holds, per round, that round's HtDs then its DtHs.
 */
int64_t oracle_rounds_simulate(const int64_t *tasks, int T, int R, const int *seq, int q, int p_htd,
                               int p_dth, int dma) {
    int n = T * R;
    int neng = dma == 2 ? 3 : 2;
    int qkind[3][2 * OMAXN], qtask[3][2 * OMAXN], qlen[3] = {0, 0, 0}, qhead[3] = {0, 0, 0};
    int run_kind[3] = {-1, -1, -1}, run_task[3] = {-1, -1, -1};
    int64_t left[3] = {0, 0, 0}, rate[3], est[3];
    unsigned char done[3][OMAXN];
    memset(done, 0, sizeof(done));
    if (dma == 2) {
        for (int j = 0; j < n; ++j)
            for (int e = 0; e < 3; ++e) { qkind[e][qlen[e]] = e; qtask[e][qlen[e]++] = seq[j]; }
    } else {
        for (int r = 0; r < R; ++r) {
            for (int i = 0; i < T; ++i) { qkind[0][qlen[0]] = K_HTD; qtask[0][qlen[0]++] = seq[r * T + i]; }
            for (int i = 0; i < T; ++i) { qkind[0][qlen[0]] = K_DTH; qtask[0][qlen[0]++] = seq[r * T + i]; }
        }
        for (int j = 0; j < n; ++j) { qkind[1][qlen[1]] = K_KER; qtask[1][qlen[1]++] = seq[j]; }
    }
    int64_t t = 0, total = 0;
    for (;;) {
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 && left[e] == 0) {
                    done[run_kind[e]][run_task[e]] = 1;
                    if (t > total) total = t;
                    run_kind[e] = -1;
                    changed = 1;
                }
            }
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 || qhead[e] >= qlen[e]) continue;
                int k = qkind[e][qhead[e]], x = qtask[e][qhead[e]];
                int ready = k == K_HTD ? (x % R == 0 || done[K_DTH][x - 1])
                          : k == K_KER ? done[K_HTD][x] : done[K_KER][x];
                if (!ready) continue;
                qhead[e]++;
                run_kind[e] = k;
                run_task[e] = x;
                left[e] = tasks[x * 3 + k] * (k == K_KER ? 1 : q);
                changed = 1;
            }
        }
        int busy = 0, hbusy = 0, dbusy = 0;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            busy = 1;
            if (run_kind[e] == K_HTD) hbusy = 1;
            if (run_kind[e] == K_DTH) dbusy = 1;
        }
        if (!busy) break;
        int64_t delta = INT64_MAX;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            int k = run_kind[e];
            rate[e] = k == K_KER ? 1 : (hbusy && dbusy ? (k == K_HTD ? p_htd : p_dth) : q);
            est[e] = ceil_div(left[e], rate[e]);
            if (est[e] < delta) delta = est[e];
        }
        t += delta;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            left[e] = est[e] == delta ? 0 : left[e] - rate[e] * delta;
        }
    }
    return total;
}

typedef struct {
    const int64_t *tasks;
    int T, R, q, p_htd, p_dth, dma;
    uint64_t lo, hi;
    int64_t *out;
} rjob_t;

static void *rounds_worker(void *arg) {
    rjob_t *j = (rjob_t *)arg;
    uint64_t tf = 1;
    for (int i = 2; i <= j->T; ++i) tf *= (uint64_t)i;
    int seq[OMAXN];
    for (uint64_t rk = j->lo; rk < j->hi; ++rk) {
        uint64_t rem = rk;
        for (int r = j->R - 1; r >= 0; --r) {
            int perm[OMAXN];
            decode_rank(j->T, rem % tf, perm);
            rem /= tf;
            for (int i = 0; i < j->T; ++i) seq[r * j->T + i] = perm[i] * j->R + r;
        }
        j->out[rk] = oracle_rounds_simulate(j->tasks, j->T, j->R, seq, j->q, j->p_htd, j->p_dth, j->dma);
    }
    return NULL;
}

/* T of every NoReorder ordering, out[rank] (rank: mixed radix T!, round 0
 * most significant), on nthreads threads. */
int oracle_rounds_times(const int64_t *tasks, int T, int R, int q, int p_htd, int p_dth, int dma,
                        int nthreads, int64_t *out) {
    if (T < 1 || R < 1 || T * R > OMAXN || nthreads < 1) return -1;
    uint64_t tf = 1, count = 1;
    for (int i = 2; i <= T; ++i) tf *= (uint64_t)i;
    for (int r = 0; r < R; ++r) count *= tf;
    rjob_t *jobs = (rjob_t *)calloc((size_t)nthreads, sizeof(rjob_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t per = (count + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int i = 0; i < nthreads; ++i) {
        rjob_t *j = &jobs[i];
        j->tasks = tasks; j->T = T; j->R = R; j->q = q; j->p_htd = p_htd; j->p_dth = p_dth; j->dma = dma;
        j->lo = (uint64_t)i * per < count ? (uint64_t)i * per : count;
        j->hi = j->lo + per < count ? j->lo + per : count;
        j->out = out;
        pthread_create(&th[i], NULL, rounds_worker, j);
    }
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------ device-memory limit */
/*
 * Transcription of oracle/memory.py: task x holds mem[x] bytes from the start
 * of its HtD to the end of its DtH, at most cap bytes at once.  Two DMA
 * engines: the HtD at the head of its queue waits until its buffers fit.  One
 * DMA engine: the ordering is cut greedily into consecutive sub-groups whose
 * buffers fit together, each launched as its HtDs then its DtHs.
 * Returns the total time, or -1 if commands were left unstarted.
 */
int64_t oracle_mem_simulate(const int64_t *tasks, const int64_t *mem, int n, int64_t cap,
                            const int *order, int q, int p_htd, int p_dth, int dma) {
    int neng = dma == 2 ? 3 : 2;
    int qkind[3][2 * OMAXN], qtask[3][2 * OMAXN], qlen[3] = {0, 0, 0}, qhead[3] = {0, 0, 0};
    int run_kind[3] = {-1, -1, -1}, run_task[3] = {-1, -1, -1};
    int64_t left[3] = {0, 0, 0}, rate[3], est[3];
    unsigned char done[3][OMAXN];
    memset(done, 0, sizeof(done));
    if (dma == 2) {
        for (int j = 0; j < n; ++j)
            for (int e = 0; e < 3; ++e) { qkind[e][qlen[e]] = e; qtask[e][qlen[e]++] = order[j]; }
    } else {
        int b = 0;
        while (b < n) {
            int e = b;
            int64_t held = 0;
            while (e < n && (e == b || held + mem[order[e]] <= cap)) held += mem[order[e++]];
            for (int i = b; i < e; ++i) { qkind[0][qlen[0]] = K_HTD; qtask[0][qlen[0]++] = order[i]; }
            for (int i = b; i < e; ++i) { qkind[0][qlen[0]] = K_DTH; qtask[0][qlen[0]++] = order[i]; }
            b = e;
        }
        for (int j = 0; j < n; ++j) { qkind[1][qlen[1]] = K_KER; qtask[1][qlen[1]++] = order[j]; }
    }
    int64_t t = 0, total = 0, held = 0;
    for (;;) {
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 && left[e] == 0) {
                    done[run_kind[e]][run_task[e]] = 1;
                    if (run_kind[e] == K_DTH) held -= mem[run_task[e]];
                    if (t > total) total = t;
                    run_kind[e] = -1;
                    changed = 1;
                }
            }
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 || qhead[e] >= qlen[e]) continue;
                int k = qkind[e][qhead[e]], x = qtask[e][qhead[e]];
                int ready = k == K_HTD ? held + mem[x] <= cap : k == K_KER ? done[K_HTD][x] : done[K_KER][x];
                if (!ready) continue;
                qhead[e]++;
                if (k == K_HTD) held += mem[x];
                run_kind[e] = k;
                run_task[e] = x;
                left[e] = tasks[x * 3 + k] * (k == K_KER ? 1 : q);
                changed = 1;
            }
        }
        int busy = 0, hbusy = 0, dbusy = 0;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            busy = 1;
            if (run_kind[e] == K_HTD) hbusy = 1;
            if (run_kind[e] == K_DTH) dbusy = 1;
        }
        if (!busy) break;
        int64_t delta = INT64_MAX;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            int k = run_kind[e];
            rate[e] = k == K_KER ? 1 : (hbusy && dbusy ? (k == K_HTD ? p_htd : p_dth) : q);
            est[e] = ceil_div(left[e], rate[e]);
            if (est[e] < delta) delta = est[e];
        }
        t += delta;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            left[e] = est[e] == delta ? 0 : left[e] - rate[e] * delta;
        }
    }
    for (int e = 0; e < neng; ++e)
        if (qhead[e] < qlen[e]) return -1;
    return total;
}

typedef struct {
    const int64_t *tasks, *mem;
    int n, q, p_htd, p_dth, dma;
    int64_t cap;
    uint64_t lo, hi, base;
    int64_t *out;
} mjob_t;

static void *mem_worker(void *arg) {
    mjob_t *j = (mjob_t *)arg;
    int perm[OMAXN];
    if (j->lo >= j->hi) return NULL;
    decode_rank(j->n, j->lo, perm);
    for (uint64_t rk = j->lo; rk < j->hi; ++rk) {
        j->out[rk - j->base] = oracle_mem_simulate(j->tasks, j->mem, j->n, j->cap, perm, j->q, j->p_htd,
                                                   j->p_dth, j->dma);
        next_perm(j->n, perm);
    }
    return NULL;
}

/* T of the orderings of ranks [lo, hi) under the memory limit, out[rank - lo],
 * on nthreads threads. */
int oracle_mem_times(const int64_t *tasks, const int64_t *mem, int n, int64_t cap, int q, int p_htd,
                     int p_dth, int dma, uint64_t lo, uint64_t hi, int nthreads, int64_t *out) {
    if (n < 1 || n > OMAXN || nthreads < 1 || hi < lo) return -1;
    mjob_t *jobs = (mjob_t *)calloc((size_t)nthreads, sizeof(mjob_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t count = hi - lo, per = (count + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int i = 0; i < nthreads; ++i) {
        mjob_t *j = &jobs[i];
        j->tasks = tasks; j->mem = mem; j->n = n; j->cap = cap;
        j->q = q; j->p_htd = p_htd; j->p_dth = p_dth; j->dma = dma;
        j->lo = lo + ((uint64_t)i * per < count ? (uint64_t)i * per : count);
        j->hi = j->lo + per < hi ? j->lo + per : hi;
        j->base = lo;
        j->out = out;
        pthread_create(&th[i], NULL, mem_worker, j);
    }
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------------------------
 * Concurrent kernels (oracle/cke.py): kernel x holds units[x] of `cap` from
 * its start to its end; kernels are dispatched in launch order when their HtD
 * has ended and their units fit beside the running kernels; running kernels
 * take their solo time.  Transfers as in oracle_simulate.  Returns T. */
int64_t oracle_cke_simulate(const int64_t *tasks, const int *units, int n, int cap, const int *order, int q,
                            int p_htd, int p_dth, int dma) {
    int neng = dma == 2 ? 2 : 1; /* transfer engines: HtD, DtH (two) or one */
    int qkind[2][2 * OMAXN], qtask[2][2 * OMAXN], qlen[2] = {0, 0}, qhead[2] = {0, 0};
    int run_kind[2] = {-1, -1}, run_task[2] = {-1, -1};
    int64_t left[2] = {0, 0}, rate[2], est[2];
    int64_t kleft[OMAXN];
    unsigned char krun[OMAXN], hdone[OMAXN], kdone[OMAXN];
    memset(krun, 0, sizeof(krun));
    memset(hdone, 0, sizeof(hdone));
    memset(kdone, 0, sizeof(kdone));
    for (int j = 0; j < n; ++j) {
        if (dma == 2) {
            qkind[0][qlen[0]] = K_HTD; qtask[0][qlen[0]++] = order[j];
            qkind[1][qlen[1]] = K_DTH; qtask[1][qlen[1]++] = order[j];
        } else {
            qkind[0][qlen[0]] = K_HTD; qtask[0][qlen[0]++] = order[j];
        }
    }
    if (dma != 2)
        for (int j = 0; j < n; ++j) { qkind[0][qlen[0]] = K_DTH; qtask[0][qlen[0]++] = order[j]; }
    int khead = 0, held = 0;
    int64_t t = 0, total = 0;
    for (;;) {
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 && left[e] == 0) {
                    if (run_kind[e] == K_HTD) hdone[run_task[e]] = 1;
                    if (t > total) total = t;
                    run_kind[e] = -1;
                    changed = 1;
                }
            }
            for (int x = 0; x < n; ++x) {
                if (krun[x] && kleft[x] == 0) {
                    krun[x] = 0;
                    kdone[x] = 1;
                    held -= units[x];
                    if (t > total) total = t;
                    changed = 1;
                }
            }
            for (int e = 0; e < neng; ++e) {
                if (run_kind[e] >= 0 || qhead[e] >= qlen[e]) continue;
                int k = qkind[e][qhead[e]], x = qtask[e][qhead[e]];
                if (k == K_DTH && !kdone[x]) continue;
                qhead[e]++;
                run_kind[e] = k;
                run_task[e] = x;
                left[e] = tasks[x * 3 + k] * q;
                changed = 1;
            }
            while (khead < n && hdone[order[khead]] && held + units[order[khead]] <= cap) {
                int x = order[khead++];
                krun[x] = 1;
                kleft[x] = tasks[x * 3 + K_KER];
                held += units[x];
                changed = 1;
            }
        }
        int busy = 0, hbusy = 0, dbusy = 0;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            busy = 1;
            if (run_kind[e] == K_HTD) hbusy = 1;
            if (run_kind[e] == K_DTH) dbusy = 1;
        }
        int64_t delta = INT64_MAX;
        for (int x = 0; x < n; ++x)
            if (krun[x]) {
                busy = 1;
                if (kleft[x] < delta) delta = kleft[x];
            }
        if (!busy) break;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            rate[e] = hbusy && dbusy ? (run_kind[e] == K_HTD ? p_htd : p_dth) : q;
            est[e] = ceil_div(left[e], rate[e]);
            if (est[e] < delta) delta = est[e];
        }
        t += delta;
        for (int e = 0; e < neng; ++e) {
            if (run_kind[e] < 0) continue;
            left[e] = est[e] == delta ? 0 : left[e] - rate[e] * delta;
        }
        for (int x = 0; x < n; ++x)
            if (krun[x]) kleft[x] -= delta;
    }
    if (khead < n) return -1;
    for (int e = 0; e < neng; ++e)
        if (qhead[e] < qlen[e]) return -1;
    return total;
}

typedef struct {
    const int64_t *tasks;
    const int *units;
    int n, cap, q, p_htd, p_dth, dma;
    uint64_t lo, hi, base;
    int64_t *out;
} cjob_t;

static void *cke_worker(void *arg) {
    cjob_t *j = (cjob_t *)arg;
    int perm[OMAXN];
    if (j->lo >= j->hi) return NULL;
    decode_rank(j->n, j->lo, perm);
    for (uint64_t rk = j->lo; rk < j->hi; ++rk) {
        j->out[rk - j->base] = oracle_cke_simulate(j->tasks, j->units, j->n, j->cap, perm, j->q, j->p_htd,
                                                   j->p_dth, j->dma);
        next_perm(j->n, perm);
    }
    return NULL;
}

/* T under the concurrent-kernel rule for the orderings of ranks [lo, hi),
 * out[rank - lo], on nthreads threads. */
int oracle_cke_times(const int64_t *tasks, const int *units, int n, int cap, int q, int p_htd, int p_dth,
                     int dma, uint64_t lo, uint64_t hi, int nthreads, int64_t *out) {
    if (n < 1 || n > OMAXN || nthreads < 1 || hi < lo) return -1;
    cjob_t *jobs = (cjob_t *)calloc((size_t)nthreads, sizeof(cjob_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t count = hi - lo, per = (count + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int i = 0; i < nthreads; ++i) {
        cjob_t *j = &jobs[i];
        j->tasks = tasks; j->units = units; j->n = n; j->cap = cap;
        j->q = q; j->p_htd = p_htd; j->p_dth = p_dth; j->dma = dma;
        j->lo = lo + ((uint64_t)i * per < count ? (uint64_t)i * per : count);
        j->hi = j->lo + per < hi ? j->lo + per : hi;
        j->base = lo;
        j->out = out;
        pthread_create(&th[i], NULL, cke_worker, j);
    }
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(jobs);
    free(th);
    return 0;
}
