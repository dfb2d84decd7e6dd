/*
 * Host model of the chained scan with decoupled look-back that the digit-binning
 * kernel runs over its tiles (Onesweep, Section 3: "Chained scan digit-binning
 * kernel", Figures 6 and 7; the look-back itself is the decoupled look-back of
 * Section 2, Figure 2).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/: only tests/ build and run
 * it. It shares no code with the HIP library and includes none of its headers.
 *
 * What is modelled. A tile owns one status word per digit, a 2-bit status above
 * a 30-bit value (Figure 6): N (0, nothing yet), L (1, the tile's own count of
 * the digit) or G (2, the inclusive prefix over every tile up to and including
 * this one). Tiles are taken in increasing order from a shared ticket. A tile
 *   1. publishes its local count as L (the first tile may publish it as G at
 *      once, since its count is already an inclusive prefix);
 *   2. walks backwards over its predecessors' words, W at a time: N means
 *      "wait and read again", L adds the value and goes on, G adds the value and
 *      ends the walk; reaching the front of the array also ends it;
 *   3. publishes G with (sum of the walk) + (own count); the sum is the tile's
 *      exclusive prefix.
 * With W = 1 this is the walk the paper describes; W > 1 reads several
 * predecessors per round trip and consumes them in order up to the first N.
 *
 * Three drivers exercise the same per-tile steps:
 *   - lookback_model_schedule: one host thread replays a given order of single
 *     steps (a step is one publish or one read of one predecessor word), and
 *     records the status array after every step; the tests replay the
 *     timeline the paper walks through beside Figure 7;
 *   - lookback_model_random: one host thread picks, with a seeded generator,
 *     which in-flight tile takes the next step, with at most `in_flight` tiles
 *     holding tickets, and may hold one tile back for a long time;
 *   - lookback_model_threads: real host threads act as workgroups, take
 *     tickets, sleep for seeded random times between steps, and one tile can be
 *     stalled before it publishes anything. Built with -fsanitize=thread by the
 *     tests. A wait that exceeds `spin_limit` reads of not-ready words stops
 *     the model with an error instead of hanging.
 * Every driver writes the final status words and each tile's exclusive
 * prefixes, which the tests compare with a sequential exclusive scan of the
 * counts.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <sched.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define LB_N 0u
#define LB_L 1u
#define LB_G 2u
#define LB_VALUE_MASK 0x3FFFFFFFu

static uint32_t lb_word(uint32_t status, uint32_t value) { return (status << 30) | (value & LB_VALUE_MASK); }
static uint32_t lb_status(uint32_t w) { return w >> 30; }
static uint32_t lb_value(uint32_t w) { return w & LB_VALUE_MASK; }

/* Step results. */
enum { LB_PROGRESS = 0, LB_BLOCKED = 1, LB_DONE = 2 };

/* Per (tile, digit) walk state. */
typedef struct {
    int phase;        /* 0: nothing published; 1: local count published, walking; 2: done */
    int64_t next;     /* the predecessor the walk reads next */
    uint64_t sum;     /* values consumed so far */
} lb_walk;

typedef struct {
    int tiles, digits, window, first_publishes_g;
    const uint32_t *counts;     /* [tiles][digits] */
    _Atomic uint32_t *status;   /* [tiles][digits] */
    uint64_t *exclusive;        /* [tiles][digits] */
} lb_model;

static uint32_t lb_load(const lb_model *m, int64_t tile, int d) {
    return atomic_load_explicit(&m->status[(size_t)tile * m->digits + d], memory_order_relaxed);
}

static void lb_store(lb_model *m, int64_t tile, int d, uint32_t w) {
    atomic_store_explicit(&m->status[(size_t)tile * m->digits + d], w, memory_order_relaxed);
}

/*
 * One step of tile t's chained scan for digit d: publish the local count, or
 * read up to `window` predecessor words (one round trip) and consume them in
 * order; a walk that ends publishes G in the same step.
 */
static int lb_step(lb_model *m, int64_t t, int d, lb_walk *w) {
    const uint32_t count = m->counts[(size_t)t * m->digits + d];
    if (w->phase == 2) return LB_DONE;
    if (w->phase == 0) {
        w->phase = 1;
        w->next = t - 1;
        w->sum = 0;
        if (t == 0 && m->first_publishes_g) {
            lb_store(m, t, d, lb_word(LB_G, count));
            m->exclusive[(size_t)t * m->digits + d] = 0;
            w->phase = 2;
            return LB_DONE;
        }
        lb_store(m, t, d, lb_word(LB_L, count));
        return LB_PROGRESS;
    }
    int found = w->next < 0;  /* the front of the array: the prefix before tile 0 is 0 */
    int consumed = 0;
    if (!found) {
        uint32_t seen[64];
        int k = m->window < 64 ? m->window : 64;
        for (int i = 0; i < k; i++)
            seen[i] = w->next - i >= 0 ? lb_load(m, w->next - i, d) : lb_word(LB_G, 0);
        for (int i = 0; i < k && !found; i++) {
            const uint32_t s = lb_status(seen[i]);
            if (s == LB_N) break;
            w->sum += lb_value(seen[i]);
            consumed++;
            found = s == LB_G;
        }
        w->next -= consumed;
    }
    if (!found) return consumed ? LB_PROGRESS : LB_BLOCKED;
    m->exclusive[(size_t)t * m->digits + d] = w->sum;
    lb_store(m, t, d, lb_word(LB_G, (uint32_t)(w->sum + count)));
    w->phase = 2;
    return LB_DONE;
}

static void lb_init(lb_model *m, const uint32_t *counts, int tiles, int digits, int window,
                    int first_publishes_g, _Atomic uint32_t *status, uint64_t *exclusive) {
    m->tiles = tiles;
    m->digits = digits;
    m->window = window < 1 ? 1 : window;
    m->first_publishes_g = first_publishes_g;
    m->counts = counts;
    m->status = status;
    m->exclusive = exclusive;
    for (size_t i = 0; i < (size_t)tiles * digits; i++) {
        atomic_init(&status[i], lb_word(LB_N, 0));
        exclusive[i] = UINT64_MAX;
    }
}

static void lb_copy_out(const lb_model *m, uint32_t *status_out, uint64_t *exclusive_out) {
    for (size_t i = 0; i < (size_t)m->tiles * m->digits; i++) {
        if (status_out) status_out[i] = atomic_load_explicit(&m->status[i], memory_order_relaxed);
        if (exclusive_out) exclusive_out[i] = m->exclusive[i];
    }
}

/* SplitMix64 (Steele, Lea and Flood, 2014) as the model's scheduling randomness. */
static uint64_t lb_rand(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/*
 * Replays `steps` single steps of one digit (digits = 1): schedule[i] names the
 * tile that moves. snapshots[i * tiles + t] receives tile t's status word after
 * step i, and results[i] the step's outcome (LB_PROGRESS, LB_BLOCKED, LB_DONE).
 * partial[i * tiles + t] holds the sum a walking tile has consumed so far.
 * Returns 0, or -1 for invalid arguments.
 */
int lookback_model_schedule(const uint32_t *counts, int tiles, int window, int first_publishes_g,
                            const int *schedule, int steps, uint32_t *snapshots, int *results,
                            uint64_t *partial, uint64_t *exclusive_out) {
    if (tiles <= 0 || steps < 0 || !counts || !schedule) return -1;
    _Atomic uint32_t *status = malloc(sizeof(*status) * (size_t)tiles);
    uint64_t *excl = malloc(sizeof(uint64_t) * (size_t)tiles);
    lb_walk *walk = calloc((size_t)tiles, sizeof(lb_walk));
    if (!status || !excl || !walk) {
        free(status); free(excl); free(walk);
        return -1;
    }
    lb_model m;
    lb_init(&m, counts, tiles, 1, window, first_publishes_g, status, excl);
    int rc = 0;
    for (int i = 0; i < steps; i++) {
        const int t = schedule[i];
        if (t < 0 || t >= tiles) { rc = -1; break; }
        const int r = lb_step(&m, t, 0, &walk[t]);
        if (results) results[i] = r;
        for (int u = 0; u < tiles; u++) {
            if (snapshots) snapshots[(size_t)i * tiles + u] = lb_load(&m, u, 0);
            if (partial) partial[(size_t)i * tiles + u] = walk[u].sum;
        }
    }
    lb_copy_out(&m, NULL, exclusive_out);
    free(status); free(excl); free(walk);
    return rc;
}

/*
 * Seeded random interleaving on one host thread. Tickets are taken in order;
 * at most `in_flight` tiles hold one at a time (a new ticket is taken when a
 * tile finishes). Each step picks a random in-flight tile and a random digit of
 * it that is not done. The tile `stalled_tile` (or -1) takes no step until
 * `stall_steps` other steps have run. `spin_limit` bounds the number of steps
 * that find only not-ready words; exceeding it returns 1 (a wait that would
 * not end). Returns 0 on success, -1 for invalid arguments.
 * stats[0] = steps taken, stats[1] = blocked steps, stats[2] = largest number
 * of predecessor words a single (tile, digit) walk consumed.
 */
int lookback_model_random(const uint32_t *counts, int tiles, int digits, int window,
                          int first_publishes_g, int in_flight, uint64_t seed, int stalled_tile,
                          long stall_steps, long spin_limit, uint32_t *status_out,
                          uint64_t *exclusive_out, uint64_t *stats) {
    if (tiles <= 0 || digits <= 0 || in_flight <= 0 || !counts) return -1;
    const size_t cells = (size_t)tiles * digits;
    _Atomic uint32_t *status = malloc(sizeof(*status) * cells);
    uint64_t *excl = malloc(sizeof(uint64_t) * cells);
    lb_walk *walk = calloc(cells, sizeof(lb_walk));
    int *active = malloc(sizeof(int) * (size_t)in_flight);
    int *left = calloc((size_t)tiles, sizeof(int));
    if (!status || !excl || !walk || !active || !left) {
        free(status); free(excl); free(walk); free(active); free(left);
        return -1;
    }
    lb_model m;
    lb_init(&m, counts, tiles, digits, window, first_publishes_g, status, excl);
    uint64_t rng = seed;
    int next_ticket = 0, nactive = 0, rc = 0;
    long steps = 0, blocked = 0, blocked_run = 0;
    uint64_t longest = 0;
    while (next_ticket < tiles || nactive > 0) {
        while (nactive < in_flight && next_ticket < tiles) {
            left[next_ticket] = digits;
            active[nactive++] = next_ticket++;
        }
        int pick = (int)(lb_rand(&rng) % (uint64_t)nactive);
        int t = active[pick];
        if (t == stalled_tile && steps < stall_steps) {
            if (nactive == 1) { /* only the stalled tile is left: time passes */
                steps++;
                continue;
            }
            pick = (pick + 1) % nactive;
            t = active[pick];
        }
        /* a random digit of tile t that is not done */
        int d = (int)(lb_rand(&rng) % (uint64_t)digits);
        while (walk[(size_t)t * digits + d].phase == 2) d = (d + 1) % digits;
        lb_walk *w = &walk[(size_t)t * digits + d];
        const int r = lb_step(&m, t, d, w);
        steps++;
        if (r == LB_BLOCKED) {
            blocked++;
            if (++blocked_run > spin_limit) { rc = 1; break; }
        } else {
            blocked_run = 0;
        }
        if (r == LB_DONE) {
            const uint64_t walked = (uint64_t)(t - 1 - (w->next < -1 ? -1 : w->next));
            if (t > 0 && walked > longest) longest = walked;
            if (--left[t] == 0) active[pick] = active[--nactive];
        }
    }
    if (stats) {
        stats[0] = (uint64_t)steps;
        stats[1] = (uint64_t)blocked;
        stats[2] = longest;
    }
    lb_copy_out(&m, status_out, exclusive_out);
    free(status); free(excl); free(walk); free(active); free(left);
    return rc;
}

/* ------------------------------------------------------------ threaded driver */

typedef struct {
    lb_model *m;
    _Atomic int *ticket;
    _Atomic int *error;
    _Atomic long *blocked;
    uint64_t seed;
    int max_delay_us;
    int stalled_tile;
    int stall_us;
    long spin_limit;
} lb_thread_arg;

static void lb_sleep_us(int us) {
    if (us <= 0) {
        sched_yield();
        return;
    }
    struct timespec ts = {us / 1000000, (long)(us % 1000000) * 1000L};
    nanosleep(&ts, NULL);
}

static void *lb_worker(void *p) {
    lb_thread_arg *a = p;
    lb_model *m = a->m;
    uint64_t rng = a->seed;
    lb_walk *walk = calloc((size_t)m->digits, sizeof(lb_walk));
    int *order = malloc(sizeof(int) * (size_t)m->digits);
    if (!walk || !order) {
        atomic_store(a->error, 2);
        free(walk); free(order);
        return NULL;
    }
    for (;;) {
        const int t = atomic_fetch_add_explicit(a->ticket, 1, memory_order_relaxed);
        if (t >= m->tiles || atomic_load_explicit(a->error, memory_order_relaxed)) break;
        memset(walk, 0, sizeof(lb_walk) * (size_t)m->digits);
        /* ranking the tile takes a while; a stalled tile takes much longer */
        lb_sleep_us(a->max_delay_us ? (int)(lb_rand(&rng) % (uint64_t)a->max_delay_us) : 0);
        if (t == a->stalled_tile) lb_sleep_us(a->stall_us);
        /* publish every digit's local count, digits in a random order */
        for (int d = 0; d < m->digits; d++) order[d] = d;
        for (int d = m->digits - 1; d > 0; d--) {
            const int j = (int)(lb_rand(&rng) % (uint64_t)(d + 1));
            const int x = order[d];
            order[d] = order[j];
            order[j] = x;
        }
        for (int i = 0; i < m->digits; i++) lb_step(m, t, order[i], &walk[order[i]]);
        lb_sleep_us(a->max_delay_us ? (int)(lb_rand(&rng) % (uint64_t)a->max_delay_us) : 0);
        /* the look-back of every digit; a not-ready word is read again */
        for (int i = 0; i < m->digits; i++) {
            const int d = order[i];
            long spins = 0;
            int r;
            while ((r = lb_step(m, t, d, &walk[d])) != LB_DONE) {
                if (r == LB_BLOCKED) {
                    atomic_fetch_add_explicit(a->blocked, 1, memory_order_relaxed);
                    if (++spins > a->spin_limit) {
                        atomic_store(a->error, 1);
                        break;
                    }
                    sched_yield();
                }
            }
            if (r != LB_DONE) break;
        }
        if (atomic_load_explicit(a->error, memory_order_relaxed)) break;
    }
    free(walk);
    free(order);
    return NULL;
}

/*
 * `threads` host threads run the chained scan over `tiles` tiles of `digits`
 * digits. Each thread sleeps a seeded random time below `max_delay_us` after
 * taking a ticket and again after publishing; `stalled_tile` (or -1) sleeps
 * `stall_us` more before it publishes anything. A (tile, digit) walk that
 * reads not-ready words more than `spin_limit` times in a row stops every
 * thread and the call returns 1. Returns 0 on success, -1 for invalid
 * arguments, 2 when memory could not be allocated. stats[0] = reads that found
 * a not-ready word.
 */
int lookback_model_threads(const uint32_t *counts, int tiles, int digits, int threads, int window,
                           int first_publishes_g, uint64_t seed, int max_delay_us, int stalled_tile,
                           int stall_us, long spin_limit, uint32_t *status_out,
                           uint64_t *exclusive_out, uint64_t *stats) {
    if (tiles <= 0 || digits <= 0 || threads <= 0 || threads > 256 || !counts) return -1;
    const size_t cells = (size_t)tiles * digits;
    _Atomic uint32_t *status = malloc(sizeof(*status) * cells);
    uint64_t *excl = malloc(sizeof(uint64_t) * cells);
    pthread_t *tid = malloc(sizeof(pthread_t) * (size_t)threads);
    lb_thread_arg *args = malloc(sizeof(lb_thread_arg) * (size_t)threads);
    if (!status || !excl || !tid || !args) {
        free(status); free(excl); free(tid); free(args);
        return 2;
    }
    lb_model m;
    lb_init(&m, counts, tiles, digits, window, first_publishes_g, status, excl);
    _Atomic int ticket, error;
    _Atomic long blocked;
    atomic_init(&ticket, 0);
    atomic_init(&error, 0);
    atomic_init(&blocked, 0);
    int started = 0;
    for (int i = 0; i < threads; i++) {
        uint64_t s = seed + 0x1000u * (uint64_t)(i + 1);
        args[i] = (lb_thread_arg){&m, &ticket, &error, &blocked, lb_rand(&s), max_delay_us,
                                  stalled_tile, stall_us, spin_limit};
        if (pthread_create(&tid[i], NULL, lb_worker, &args[i]) != 0) {
            atomic_store(&error, 2);
            break;
        }
        started++;
    }
    for (int i = 0; i < started; i++) pthread_join(tid[i], NULL);
    lb_copy_out(&m, status_out, exclusive_out);
    if (stats) stats[0] = (uint64_t)atomic_load(&blocked);
    const int rc = atomic_load(&error);
    free(status); free(excl); free(tid); free(args);
    return rc;
}

#ifdef LOOKBACK_MODEL_MAIN
/*
 * Stand-alone driver for the thread-sanitizer build:
 *   lookback_model tiles digits threads window first_g seed max_delay_us stalled stall_us
 * Runs the threaded model and checks it against a sequential scan of seeded
 * counts; exits 0 when every exclusive prefix and final word is right.
 */
#include <stdio.h>
int main(int argc, char **argv) {
    if (argc != 10) {
        fprintf(stderr, "usage: %s tiles digits threads window first_g seed max_delay_us "
                        "stalled_tile stall_us\n", argv[0]);
        return 64;
    }
    const int tiles = atoi(argv[1]), digits = atoi(argv[2]), threads = atoi(argv[3]);
    const int window = atoi(argv[4]), first_g = atoi(argv[5]);
    uint64_t seed = strtoull(argv[6], NULL, 10);
    const int delay = atoi(argv[7]), stalled = atoi(argv[8]), stall_us = atoi(argv[9]);
    const size_t cells = (size_t)tiles * digits;
    uint32_t *counts = malloc(sizeof(uint32_t) * cells), *st = malloc(sizeof(uint32_t) * cells);
    uint64_t *ex = malloc(sizeof(uint64_t) * cells), stats[1];
    if (!counts || !st || !ex) return 65;
    uint64_t s = seed;
    for (size_t i = 0; i < cells; i++) counts[i] = (uint32_t)(lb_rand(&s) % 200u);
    const int rc = lookback_model_threads(counts, tiles, digits, threads, window, first_g, seed,
                                          delay, stalled, stall_us, 1L << 40, st, ex, stats);
    if (rc != 0) {
        fprintf(stderr, "model returned %d\n", rc);
        return 1;
    }
    for (int d = 0; d < digits; d++) {
        uint64_t run = 0;
        for (int t = 0; t < tiles; t++) {
            const size_t i = (size_t)t * digits + d;
            if (ex[i] != run || st[i] != lb_word(LB_G, (uint32_t)(run + counts[i]))) {
                fprintf(stderr, "tile %d digit %d: exclusive %llu (want %llu), word %08x\n", t, d,
                        (unsigned long long)ex[i], (unsigned long long)run, st[i]);
                return 1;
            }
            run += counts[i];
        }
    }
    printf("ok: %d tiles x %d digits, %d threads, window %d, %llu not-ready reads\n", tiles,
           digits, threads, window, (unsigned long long)stats[0]);
    free(counts); free(st); free(ex);
    return 0;
}
#endif
