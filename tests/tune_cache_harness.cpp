// Host-only checks of the segmented tuner's cache file format
// (paper_1808_10292_amd/csrc/tune_cache.h).  argv[1] is a scratch directory.
// Exit status 0 and a final "OK" line mean every check passed.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "../paper_1808_10292_amd/csrc/tune_cache.h"

using rsort::TuneEntry;
using rsort::TuneKey;

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                                      \
        }                                                                 \
    } while (0)

static TuneEntry entry(const char* arch, int kt, int pl, int lk, int ls, uint32_t split, int srt,
                       int tile, int launch, double ms)
{
    TuneEntry e;
    memset(&e, 0, sizeof e);
    rsort::set_tune_arch(&e.key, arch);
    e.key.key_type = kt;
    e.key.payload = pl;
    e.key.log2_keys = lk;
    e.key.log2_segs = ls;
    e.split = split;
    e.small_sort = srt;
    e.tile_threads = tile;
    e.launch = launch;
    e.ms = ms;
    return e;
}

static bool same_entry(const TuneEntry& a, const TuneEntry& b)
{
    return rsort::same_tune_key(a.key, b.key) && a.split == b.split && a.small_sort == b.small_sort &&
           a.tile_threads == b.tile_threads && a.launch == b.launch && a.ms == b.ms;
}

static void write_file(const std::string& path, const std::string& text)
{
    FILE* f = fopen(path.c_str(), "w");
    CHECK(f != nullptr);
    CHECK(fwrite(text.data(), 1, text.size(), f) == text.size());
    CHECK(fclose(f) == 0);
}

int main(int argc, char** argv)
{
    CHECK(argc == 2);
    const std::string dir = argv[1];

    // ceiling of log2
    CHECK(rsort::ceil_log2(0) == 0 && rsort::ceil_log2(1) == 0 && rsort::ceil_log2(2) == 1);
    CHECK(rsort::ceil_log2(3) == 2 && rsort::ceil_log2(4096) == 12 && rsort::ceil_log2(4097) == 13);
    CHECK(rsort::ceil_log2(~0ull) == 64 && rsort::ceil_log2((1ull << 63) + 1) == 64);

    // architecture name: the part before the first ':', at most 31 characters
    TuneKey k;
    rsort::set_tune_arch(&k, "gfx950:sramecc+:xnack-");
    CHECK(strcmp(k.arch, "gfx950") == 0);
    rsort::set_tune_arch(&k, "gfx950");
    CHECK(strcmp(k.arch, "gfx950") == 0);
    rsort::set_tune_arch(&k, "abcdefghijklmnopqrstuvwxyz0123456789");
    CHECK(strlen(k.arch) == 31 && strncmp(k.arch, "abcdefghijklmnopqrstuvwxyz01234", 31) == 0);

    // the written line parses back to the same entry (times to 6 decimals)
    const TuneEntry a = entry("gfx950", 0, 0, 26, 12, 8192, 0, 512, 0, 0.722);
    const TuneEntry b = entry("gfx950", 0, 1, 26, 12, 4096, 1, 1024, 1, 3.125);
    const TuneEntry c = entry("gfx942", 0, 0, 26, 12, 1024, 2, 256, 0, 1.5);
    TuneEntry got;
    const std::string la = rsort::format_tune_entry(a);
    CHECK(la == "{\"arch\": \"gfx950\", \"key_type\": 0, \"payload\": 0, \"log2_keys\": 26, "
                "\"log2_segs\": 12, \"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, "
                "\"launch\": 0, \"ms\": 0.722000}");
    CHECK(rsort::parse_tune_entry(la.c_str(), &got) && same_entry(got, a));
    CHECK(rsort::parse_tune_entry(("  " + la + "\r\n").c_str(), &got) && same_entry(got, a));

    // anything else is refused, and leaves the output alone
    const TuneEntry keep = got;
    const char* bad[] = {
        "",
        "{}",
        "{\"arch\": \"gfx950\", \"key_type\": 0}",
        "{\"arch\": \"gfx950\", \"key_type\": 0, \"payload\": 0, \"log2_keys\": 26, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": 0.7",
        "{\"arch\": \"gfx950\", \"key_type\": 0, \"payload\": 0, \"log2_keys\": 26, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": 0.7} x",
        "{\"arch\": \"gfx950\", \"key_type\": 0, \"payload\": 2, \"log2_keys\": 26, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": 0.7}",
        "{\"arch\": \"gfx950\", \"key_type\": 0, \"payload\": 0, \"log2_keys\": 65, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": 0.7}",
        "{\"arch\": \"gfx950\", \"key_type\": 0, \"payload\": 0, \"log2_keys\": 26, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": -1.0}",
        "{\"arch\": \"gfx:950\", \"key_type\": 0, \"payload\": 0, \"log2_keys\": 26, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": 0.7}",
        "{\"arch\": \"gfx950\", \"payload\": 0, \"key_type\": 0, \"log2_keys\": 26, \"log2_segs\": 12, "
        "\"split\": 8192, \"small_sort\": 0, \"tile_threads\": 512, \"launch\": 0, \"ms\": 0.7}",
    };
    for (const char* s : bad) {
        got = keep;
        CHECK(!rsort::parse_tune_entry(s, &got));
        CHECK(same_entry(got, keep));
    }

    // keys differ in every field
    TuneKey kk = a.key;
    CHECK(rsort::same_tune_key(kk, a.key));
    kk.key_type = 1;
    CHECK(!rsort::same_tune_key(kk, a.key));
    kk = a.key;
    kk.payload = 1;
    CHECK(!rsort::same_tune_key(kk, a.key));
    kk = a.key;
    kk.log2_keys = 25;
    CHECK(!rsort::same_tune_key(kk, a.key));
    kk = a.key;
    kk.log2_segs = 11;
    CHECK(!rsort::same_tune_key(kk, a.key));
    CHECK(!rsort::same_tune_key(c.key, a.key));

    // no file, or no line with the key: no entry
    const std::string path = dir + "/tune.jsonl";
    CHECK(!rsort::lookup_tune_entry(path.c_str(), a.key, &got));
    CHECK(!rsort::lookup_tune_entry(nullptr, a.key, &got));
    CHECK(!rsort::lookup_tune_entry("", a.key, &got));
    CHECK(!rsort::append_tune_entry((dir + "/missing/tune.jsonl").c_str(), a));

    // appended lines: the last one with the key wins; damaged lines, a line
    // longer than the reader's buffer that ends in a valid entry, and a last
    // line without its newline are skipped
    CHECK(rsort::append_tune_entry(path.c_str(), a));
    CHECK(rsort::lookup_tune_entry(path.c_str(), a.key, &got) && same_entry(got, a));
    CHECK(!rsort::lookup_tune_entry(path.c_str(), b.key, &got));
    TuneEntry a2 = a;
    a2.split = 4096;
    a2.ms = 0.5;
    CHECK(rsort::append_tune_entry(path.c_str(), c));
    CHECK(rsort::append_tune_entry(path.c_str(), a2));
    CHECK(rsort::append_tune_entry(path.c_str(), b));
    CHECK(rsort::lookup_tune_entry(path.c_str(), a.key, &got) && same_entry(got, a2));
    CHECK(rsort::lookup_tune_entry(path.c_str(), b.key, &got) && same_entry(got, b));
    CHECK(rsort::lookup_tune_entry(path.c_str(), c.key, &got) && same_entry(got, c));

    TuneEntry a3 = a;
    a3.split = 0;
    std::string text = rsort::format_tune_entry(a) + "\n";
    text += "{\"arch\": \"gfx950\", \"key_type\": 0,\n";                       // damaged
    text += std::string(600, ' ') + rsort::format_tune_entry(a3) + "\n";   // longer than the buffer
    text += "not json at all\n\n";
    text += rsort::format_tune_entry(a3);                                   // no newline
    write_file(path, text);
    CHECK(rsort::lookup_tune_entry(path.c_str(), a.key, &got) && same_entry(got, a));

    printf("OK\n");
    return 0;
}
