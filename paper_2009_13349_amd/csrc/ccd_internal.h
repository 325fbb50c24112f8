// Structures shared by the kernels and the host runtime of the CCD library.
#pragma once
#include <stdint.h>

namespace ccd {

// Device counters (uint64 each) kept in one small scratch array per context.
enum Counter : int {
    kCntCursor = 0,      // lane engine: next index into the query order
    kCntOrderFront,      // root pass: next VF slot
    kCntOrderBack,       // root pass: next EE slot (counts down from n)
    kCntRecA,            // records handed from the lane engine to the group engine
    kCntRecATake,        // group engine: next record to take
    kCntRecB,            // records handed from the group engine to the block engine
    kCntRecBTake,        // block engine: next record to take
    kCntOverflow,        // queries returned with the overflow status (scratch too small)
    kCntChecks,          // 6 counters: checks [tier 0..2][kind 0..1]
    kCntSlots = kCntChecks + 6,  // 3 counters: lane slots spent per tier (utilisation)
    kCntPool = kCntSlots + 3,    // words taken from the group -> block hand-off pool
    kCntRestart,         // group -> block hand-offs that restart at level 0 (pool full)
    kCntDeep,            // lane engine: queries handed on because a level passed depth sum 64
    kCntProbe,           // group engines: level probes run
    kCntProbeHit,        // group engines: level probes that decided the level
    kCntTail,            // single-wave groups: levels handed on after their queue drained
    kCntEnd,
};
static_assert(kCntEnd <= 64, "counters are cleared by one wavefront");

// One request of a serving launch: its queries occupy the global indices
// [base, base + n) of the launch.
struct ReqEntry {
    int64_t base;
    int64_t n;
    const double* pos;      // [24][n]
    const uint8_t* kind;    // [n] or null
    double delta;
    int64_t max_iter;
    double min_sep;
    double t_max;           // time interval [0, t_max]
    uint32_t flags;
    uint32_t default_kind;
    double* toi;
    double* t_width;
    uint8_t* hit;
    uint64_t* n_checks;
    uint8_t* status;
};

// Inputs, parameters and outputs of one batch (passed by value to kernels).
// With reqs != null the launch covers nreq requests (sorted by base) and the
// per-batch fields below other than n are unused; n is the total query count.
struct BatchArgs {
    int64_t n;
    const double* pos;          // [24][n]
    const uint8_t* kind;        // [n] or null
    const double* delta_q;      // [n] or null
    const int64_t* max_iter_q;  // [n] or null
    const double* min_sep_q;    // [n] or null
    double delta;
    int64_t max_iter;
    double min_sep;
    double t_max;               // time interval [0, t_max], 0 < t_max <= 1
    uint32_t flags;
    uint32_t default_kind;
    double* toi;
    double* t_width;
    uint8_t* hit;
    uint64_t* n_checks;
    uint8_t* status;
    unsigned long long* counters;  // [kCntEnd]
    const int64_t* order;          // [n] query order grouped by kind, or null (identity)
    const ReqEntry* reqs;          // serving: request table, or null
    int64_t nreq;
    const double* gamma;           // scene-wide gamma per axis [3], or null (per query)
};

// Storage formats of a level's boxes (group engine arenas and hand-off records).
constexpr int kFmtKey = 0;     // one packed key per box (depth sum <= 64)
constexpr int kFmtPair = 1;    // one word per sibling pair: parent key | flag << 63
constexpr int kFmtTriple = 2;  // (it, iu, iv) in three arrays of `words` entries, any depth

// A query handed from one engine to the next, at the start of a level.  The
// level's `words` storage words (three arrays of `words` for triples) follow
// the header, or (group -> block hand-offs) sit in the hand-off pool at the
// offset held in the word after the header.  A record of level 0 carries no
// boxes: its one box is the root [0,1]^3 (key 0).
struct Record {
    int64_t q;
    uint64_t N;       // box checks before this level
    double tpend;     // remembered terminal box (t_lo), +inf if none
    double wpend;     // its w(I_t)
    int32_t level;
    int32_t d[3];     // bisection depth per axis on this level
    uint32_t cnt;     // boxes on this level
    uint32_t fmt;     // kFmt* | pair split axis << 4
    uint64_t words;   // storage words per array
};
static_assert(sizeof(Record) == 64, "record header layout");
constexpr int kRecordHeaderWords = 8;

// Threads per block of the lane engine (its LDS frontier is sized per block).
constexpr int kLaneBlock = 128;

struct LaneCfg {
    int32_t capacity;          // boxes per level per lane (the LDS frontier holds 2 x capacity)
    int32_t persistent;        // 1: lanes pull queries from the cursor
    int32_t survivors;         // 1: the queries are the root pass's list in order
    int32_t pad;
    uint64_t budget;           // checks after which a query is handed on
    uint64_t* records;         // promotion records, stride record_words
    int64_t record_words;
    int64_t record_cap;
    uint8_t* record_levels;    // each record's level (at most 63), for ordering them
};

struct GroupCfg {
    int64_t capacity;          // words per level of one group's arena buffer
    int64_t lds_words;         // the first lds_words words of a packed level stay in LDS
                               // (two buffers per block, dynamic shared memory)
    uint64_t* arena;           // [groups][2][3][capacity]
    const uint64_t* in_records;
    int64_t in_record_words;
    int64_t in_record_cap;
    const uint64_t* in_pool;   // non-null: the input records' boxes are in this pool
    const int64_t* in_perm;    // non-null: the order in which the input records are taken
    int32_t in_count_idx;      // counter holding the number of input records
    int32_t in_take_idx;       // counter used to take input records
    uint64_t* out_records;     // hand-off records for the next engine (or null: none)
    int64_t out_record_words;
    int64_t out_record_cap;
    uint64_t* out_pool;        // the hand-off records' boxes (words)
    int64_t out_pool_words;
    int32_t out_count_idx;
    int32_t tier;              // 1 (group) or 2 (block), for the check counters
    int64_t tail_records;      // single-wave groups whose input records are all taken hand
                               // on a level of capacity / 16 words or more, at most this
                               // many times per launch (0: never)
};

}  // namespace ccd
