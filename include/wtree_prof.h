/*
 * wtree_prof.h -- kernel timing hooks of the wavelet-tree library.
 *
 * For benchmarks and tests.  While profiling is on, every kernel that a
 * build enqueues (wt_build, wt_build_batch) is bracketed by two hipEvents
 * recorded on the build's own stream, so the measured time is that
 * kernel's execution on that stream.  The events carry no system-scope
 * fence; still, each record between two kernels idles the stream for a
 * few microseconds, so builds timed for throughput run with profiling
 * off.  Records accumulate in a host-side list owned by the library until
 * wt_prof_enable is called again.
 */
#ifndef WTREE_PROF_H
#define WTREE_PROF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wt_prof_rec {
    char kernel[32];  /* kernel family, e.g. "level", "hist", "plan" */
    uint32_t level;   /* tree level the launch serves (0 if none) */
    uint32_t width;   /* bytes per symbol of the launch's input */
    uint64_t n;       /* symbols of the sequence(s) the launch covers */
    uint64_t bytes;   /* algorithmic bytes the launch must move (see below) */
    float ms;         /* elapsed time between the bracketing events */
} wt_prof_rec;

/*
 * Switch profiling on (1) or off (0); either way the record list is
 * cleared.  Returns WT_OK.
 */
int wt_prof_enable(int on);

/*
 * Waits for every recorded event, then copies up to `max` records into
 * out (may be NULL) and stores the number of records in *count.  The
 * algorithmic bytes of a level launch are: read the level's symbols,
 * write the next level's symbols (not on the last level), write the
 * level's bitmap words and rank directory, and, for a pass that folds in
 * the last level, that level's bitmap words instead of its symbols.
 * Returns WT_OK or WT_EDEVICE.
 */
int wt_prof_read(wt_prof_rec *out, uint64_t max, uint64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* WTREE_PROF_H */
