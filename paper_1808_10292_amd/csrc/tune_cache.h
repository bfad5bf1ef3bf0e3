// Persisted choices of the segmented sort's tuner (rsort_segmented_tune): a
// text file of one JSON object per line, each keyed by the GPU architecture,
// the key type, whether payloads move, and the batch's size class -- the
// ceiling of log2 of its total keys and of its segment count.  A lookup takes
// the last line with the key; lines that do not parse are skipped, so a
// damaged or missing file only means tuning again.  Appending writes one line
// with one call, so concurrent writers interleave whole lines.
//
// Host-only (no HIP), so that the format can be tested without a GPU.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>

namespace rsort {

struct TuneKey {
    char arch[32];   // architecture name up to its first ':' (e.g. gfx950)
    int key_type;    // rsort_key_type
    int payload;     // 1 if 32-bit payloads move with the keys
    int log2_keys;   // ceil(log2(total keys)), 0 for at most one key
    int log2_segs;   // ceil(log2(segments)), 0 for at most one segment
};

struct TuneEntry {
    TuneKey key;
    uint32_t split;   // largest segment sorted whole in LDS
    int small_sort;   // rsort_small_sort
    int tile_threads; // workgroup of the large path's tiles (256, 512, 1024)
    int launch;       // rsort_seg_launch
    double ms;        // time per sort measured when the line was written
};

inline int ceil_log2(uint64_t x)
{
    int b = 0;
    while (b < 64 && ((uint64_t)1 << b) < x) ++b;
    return b;
}

// The architecture part of a device's architecture string ("gfx950:sramecc+:xnack-").
inline void set_tune_arch(TuneKey* k, const char* gcn_arch)
{
    size_t i = 0;
    for (; gcn_arch && gcn_arch[i] && gcn_arch[i] != ':' && i + 1 < sizeof(k->arch); ++i)
        k->arch[i] = gcn_arch[i];
    k->arch[i] = 0;
}

inline bool same_tune_key(const TuneKey& a, const TuneKey& b)
{
    return strcmp(a.arch, b.arch) == 0 && a.key_type == b.key_type && a.payload == b.payload &&
           a.log2_keys == b.log2_keys && a.log2_segs == b.log2_segs;
}

inline std::string format_tune_entry(const TuneEntry& e)
{
    char buf[320];
    snprintf(buf, sizeof buf,
             "{\"arch\": \"%s\", \"key_type\": %d, \"payload\": %d, \"log2_keys\": %d, "
             "\"log2_segs\": %d, \"split\": %u, \"small_sort\": %d, \"tile_threads\": %d, "
             "\"launch\": %d, \"ms\": %.6f}",
             e.key.arch, e.key.key_type, e.key.payload, e.key.log2_keys, e.key.log2_segs,
             e.split, e.small_sort, e.tile_threads, e.launch, e.ms);
    return buf;
}

// Parses exactly the layout format_tune_entry writes (leading blanks and a
// trailing newline allowed); false for anything else.
inline bool parse_tune_entry(const char* line, TuneEntry* out)
{
    TuneEntry e;
    memset(&e, 0, sizeof e);
    int end = -1;
    const int got = sscanf(line,
                           " {\"arch\": \"%31[A-Za-z0-9_]\", \"key_type\": %d, \"payload\": %d, "
                           "\"log2_keys\": %d, \"log2_segs\": %d, \"split\": %u, "
                           "\"small_sort\": %d, \"tile_threads\": %d, \"launch\": %d, \"ms\": %lf}%n",
                           e.key.arch, &e.key.key_type, &e.key.payload, &e.key.log2_keys,
                           &e.key.log2_segs, &e.split, &e.small_sort, &e.tile_threads, &e.launch, &e.ms,
                           &end);
    if (got != 10 || end < 0) return false;
    for (const char* p = line + end; *p; ++p)
        if (*p != '\n' && *p != '\r' && *p != ' ' && *p != '\t') return false;
    if (e.key.payload != 0 && e.key.payload != 1) return false;
    if (e.key.log2_keys < 0 || e.key.log2_keys > 64 || e.key.log2_segs < 0 || e.key.log2_segs > 64)
        return false;
    if (!(e.ms >= 0.0)) return false;
    *out = e;
    return true;
}

// The last entry of the file at path with this key; false if there is none
// (or no readable file).
inline bool lookup_tune_entry(const char* path, const TuneKey& key, TuneEntry* out)
{
    FILE* f = path && *path ? fopen(path, "r") : nullptr;
    if (!f) return false;
    char line[512];
    bool found = false;
    bool whole = true;   // the buffer starts at the beginning of a line
    while (fgets(line, sizeof line, f)) {
        const bool starts = whole;
        whole = strchr(line, '\n') != nullptr;
        TuneEntry e;
        if (starts && whole && parse_tune_entry(line, &e) && same_tune_key(e.key, key)) {
            *out = e;
            found = true;
        }
    }
    fclose(f);
    return found;
}

// Appends one line; false if the file cannot be written.
inline bool append_tune_entry(const char* path, const TuneEntry& e)
{
    if (!path || !*path) return false;
    const std::string s = format_tune_entry(e) + "\n";
    FILE* f = fopen(path, "a");
    if (!f) return false;
    const bool ok = fwrite(s.data(), 1, s.size(), f) == s.size();
    return fclose(f) == 0 && ok;
}

}  // namespace rsort
