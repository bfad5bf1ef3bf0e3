/*
 * oracle/sr4.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Plain, serial, deliberately unoptimised CPU reference implementations of the
 * integer sorts studied in Gerbessiotis, "A study of integer sorting on
 * multicores" (arXiv 1808.10292).  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the GPU library never links
 * it, and the two share no source, header, table or helper.
 *
 * Every routine is written from the paper's description, in the paper's order:
 *
 *   lsd_u32 / lsd_u64  Section 3.2, "Serial radix-r radix-sort: SR4": rounds of
 *                      count-sort on lg(r)-bit digits.  Each round reads the
 *                      input once to count digit occurrences into a count array
 *                      of r entries, turns the counts into starting offsets,
 *                      then reads the input a second time and writes every key
 *                      once to its slot.  SR4 is r = 2^8 (four rounds for 32-bit
 *                      keys); PR2's serial equivalent is r = 2^16 (two rounds).
 *                      Readings (the paper does not state them): digits are
 *                      taken least-significant first, and the output loop walks
 *                      the input forward so that each round is stable -- LSD
 *                      radix sort is only correct with stable rounds.
 *   digit_counts_*     the counting loop of one round on its own.
 *   gsd_u32            Section 3.3, Algorithm 1 (GSD), steps 1-5, with the
 *                      readings listed at the function.
 *   ger_u32            Section 3.3, Algorithm 2 (GER): GSD's skeleton with a
 *                      random sample of the locally sorted blocks.
 *   gvr_u32            Section 3.3, Algorithm 3 (GVR): a random sample of the
 *                      input, splitting of the unsorted blocks by binary search
 *                      and a count sort on the bucket index, then SR4 per
 *                      bucket.  The random draws of both are caller inputs.
 *   sort_kind          signed and IEEE float keys (not in the paper): a stable
 *                      merge sort by comparison (totalOrder for floats).
 *   segmented_u32/u64  SR4 applied independently to each segment of a CSR
 *                      segment list (the batched workload).
 *
 * Payloads are an addition to the paper (which sorts keys only): an optional
 * 32-bit value travels with its key.  With a payload the stable result is
 * unique, so every sort in this file produces exactly "the" stable sort.
 *
 * All functions return 0 on success and a negative value on bad arguments or
 * allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* One count-sort round (Section 3.2): count, exclusive prefix, stable output. */

static void round_u32(const uint32_t* in, const uint32_t* vin, size_t n,
                      int shift, int width, uint32_t* out, uint32_t* vout,
                      uint64_t* count /* 2^width entries */)
{
    const uint64_t r = (uint64_t)1 << width;
    const uint32_t mask = (uint32_t)(r - 1);
    memset(count, 0, (size_t)r * sizeof(uint64_t));
    for (size_t i = 0; i < n; ++i)                         /* counting pass */
        count[(in[i] >> shift) & mask] += 1;
    uint64_t run = 0;                                      /* starting offsets */
    for (uint64_t v = 0; v < r; ++v) {
        uint64_t c = count[v];
        count[v] = run;
        run += c;
    }
    for (size_t i = 0; i < n; ++i) {                       /* output pass, forward */
        uint32_t v = (in[i] >> shift) & mask;
        uint64_t slot = count[v]++;
        out[slot] = in[i];
        if (vin) vout[slot] = vin[i];
    }
}

static void round_u64(const uint64_t* in, const uint32_t* vin, size_t n,
                      int shift, int width, uint64_t* out, uint32_t* vout,
                      uint64_t* count)
{
    const uint64_t r = (uint64_t)1 << width;
    const uint64_t mask = r - 1;
    memset(count, 0, (size_t)r * sizeof(uint64_t));
    for (size_t i = 0; i < n; ++i)
        count[(in[i] >> shift) & mask] += 1;
    uint64_t run = 0;
    for (uint64_t v = 0; v < r; ++v) {
        uint64_t c = count[v];
        count[v] = run;
        run += c;
    }
    for (size_t i = 0; i < n; ++i) {
        uint64_t v = (in[i] >> shift) & mask;
        uint64_t slot = count[v]++;
        out[slot] = in[i];
        if (vin) vout[slot] = vin[i];
    }
}

/*
 * LSD radix sort of the key bits [begin_bit, end_bit) with digits of
 * digit_bits bits (the last digit is narrower when the range is not a
 * multiple).  digit_bits = 8 is SR4; 16 is the serial form of PR2's rounds.
 * Sorting on [0, 8(d+1)) gives the array after round d of SR4.
 * keys_out/vals_out may alias keys_in/vals_in.  vals_in == NULL: keys only.
 */
int lsd_u32(const uint32_t* keys_in, const uint32_t* vals_in, size_t n,
            int digit_bits, int begin_bit, int end_bit,
            uint32_t* keys_out, uint32_t* vals_out)
{
    if (digit_bits < 1 || digit_bits > 16 || begin_bit < 0 || end_bit > 32 ||
        begin_bit > end_bit || (n && (!keys_in || !keys_out)) ||
        (vals_in && !vals_out))
        return -1;
    uint32_t* a = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t* b = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t* va = vals_in ? (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t)) : NULL;
    uint32_t* vb = vals_in ? (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t)) : NULL;
    uint64_t* count = (uint64_t*)malloc(((size_t)1 << digit_bits) * sizeof(uint64_t));
    if (!a || !b || !count || (vals_in && (!va || !vb))) {
        free(a); free(b); free(va); free(vb); free(count);
        return -2;
    }
    if (n) memcpy(a, keys_in, n * sizeof(uint32_t));
    if (vals_in && n) memcpy(va, vals_in, n * sizeof(uint32_t));
    for (int lo = begin_bit; lo < end_bit; lo += digit_bits) {
        int width = end_bit - lo < digit_bits ? end_bit - lo : digit_bits;
        round_u32(a, va, n, lo, width, b, vb, count);
        uint32_t* t = a; a = b; b = t;
        t = va; va = vb; vb = t;
    }
    if (n) memcpy(keys_out, a, n * sizeof(uint32_t));
    if (vals_in && n) memcpy(vals_out, va, n * sizeof(uint32_t));
    free(a); free(b); free(va); free(vb); free(count);
    return 0;
}

int lsd_u64(const uint64_t* keys_in, const uint32_t* vals_in, size_t n,
            int digit_bits, int begin_bit, int end_bit,
            uint64_t* keys_out, uint32_t* vals_out)
{
    if (digit_bits < 1 || digit_bits > 16 || begin_bit < 0 || end_bit > 64 ||
        begin_bit > end_bit || (n && (!keys_in || !keys_out)) ||
        (vals_in && !vals_out))
        return -1;
    uint64_t* a = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* b = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint32_t* va = vals_in ? (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t)) : NULL;
    uint32_t* vb = vals_in ? (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t)) : NULL;
    uint64_t* count = (uint64_t*)malloc(((size_t)1 << digit_bits) * sizeof(uint64_t));
    if (!a || !b || !count || (vals_in && (!va || !vb))) {
        free(a); free(b); free(va); free(vb); free(count);
        return -2;
    }
    if (n) memcpy(a, keys_in, n * sizeof(uint64_t));
    if (vals_in && n) memcpy(va, vals_in, n * sizeof(uint32_t));
    for (int lo = begin_bit; lo < end_bit; lo += digit_bits) {
        int width = end_bit - lo < digit_bits ? end_bit - lo : digit_bits;
        round_u64(a, va, n, lo, width, b, vb, count);
        uint64_t* t = a; a = b; b = t;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    if (n) memcpy(keys_out, a, n * sizeof(uint64_t));
    if (vals_in && n) memcpy(vals_out, va, n * sizeof(uint32_t));
    free(a); free(b); free(va); free(vb); free(count);
    return 0;
}

/* The counting loop of one round (Section 3.2): counts[v] = #{i : digit(x_i) = v}. */
int digit_counts_u32(const uint32_t* keys, size_t n, int shift, int width,
                     uint64_t* counts)
{
    if (width < 1 || width > 16 || shift < 0 || shift + width > 32) return -1;
    const uint32_t mask = (uint32_t)(((uint64_t)1 << width) - 1);
    memset(counts, 0, ((size_t)1 << width) * sizeof(uint64_t));
    for (size_t i = 0; i < n; ++i) counts[(keys[i] >> shift) & mask] += 1;
    return 0;
}

int digit_counts_u64(const uint64_t* keys, size_t n, int shift, int width,
                     uint64_t* counts)
{
    if (width < 1 || width > 16 || shift < 0 || shift + width > 64) return -1;
    const uint64_t mask = ((uint64_t)1 << width) - 1;
    memset(counts, 0, ((size_t)1 << width) * sizeof(uint64_t));
    for (size_t i = 0; i < n; ++i) counts[(keys[i] >> shift) & mask] += 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Segmented: SR4 on every segment [off[s], off[s+1]) independently.          */

int segmented_u32(const uint32_t* keys_in, const uint32_t* vals_in,
                  const uint64_t* offsets, size_t num_segs,
                  uint32_t* keys_out, uint32_t* vals_out)
{
    for (size_t s = 0; s < num_segs; ++s) {
        uint64_t lo = offsets[s], hi = offsets[s + 1];
        if (hi < lo) return -1;
        int rc = lsd_u32(keys_in + lo, vals_in ? vals_in + lo : NULL, hi - lo,
                         8, 0, 32, keys_out + lo, vals_in ? vals_out + lo : NULL);
        if (rc) return rc;
    }
    return 0;
}

int segmented_u64(const uint64_t* keys_in, const uint32_t* vals_in,
                  const uint64_t* offsets, size_t num_segs,
                  uint64_t* keys_out, uint32_t* vals_out)
{
    for (size_t s = 0; s < num_segs; ++s) {
        uint64_t lo = offsets[s], hi = offsets[s + 1];
        if (hi < lo) return -1;
        int rc = lsd_u64(keys_in + lo, vals_in ? vals_in + lo : NULL, hi - lo,
                         8, 0, 64, keys_out + lo, vals_in ? vals_out + lo : NULL);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* GSD, Algorithm 1 (Section 3.3).
 *
 * Readings where the paper is silent:
 *  - Block k of step 1 is [floor(k n / p), floor((k+1) n / p)); p is clamped
 *    to n so that no block is empty.
 *  - Step 2 takes, from block k of N_k sorted keys, the s = r p keys at
 *    positions ceil(j N_k / s) - 1 for j = 1..s: the last key of each of s
 *    near-equal segments, the final one being the block maximum.
 *  - Keys are compared as composites (key, g), g being the key's position in
 *    the concatenation X of the locally sorted blocks.  Because every block is
 *    sorted stably, g-order among equal keys is input order, so duplicates
 *    (which the paper defers to a discussion it does not include) are split
 *    deterministically and the result is the stable sort.
 *  - Step 3 splitter i (1 <= i <= p-1) is the (i s)-th smallest composite of
 *    the sample, 1-based.  The sample is sorted with SR4 instead of BTN; any
 *    correct sort gives the same sequence.
 *  - Step 4: X_{k,j} holds the keys e of block k with S_j < e <= S_{j+1}
 *    (S_0 = -inf, S_p = +inf): a splitter, the largest key of its sample
 *    segment, stays with the keys below it.  Its end is found by binary
 *    search.
 *  - Step 5 merges the runs X_{0,j}, ..., X_{p-1,j} with a heap, equal keys
 *    taken from the lower run first (stable).
 *
 * Outputs besides the sorted keys/values: cnt[k*p + j] = |X_{k,j}|, the
 * splitters (key, g) and, through cnt, the bucket sizes |Y_j|.
 */

static int comp_less(uint32_t ka, uint64_t ga, uint32_t kb, uint64_t gb)
{
    return ka < kb || (ka == kb && ga < gb);
}

/* heap of run heads for step 5, ordered by (key, run index) */
typedef struct { uint32_t key; uint32_t run; } head;

static int head_less(head a, head b)
{
    return a.key < b.key || (a.key == b.key && a.run < b.run);
}

static void heap_sift_down(head* h, size_t m, size_t i)
{
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, best = i;
        if (l < m && head_less(h[l], h[best])) best = l;
        if (r < m && head_less(h[r], h[best])) best = r;
        if (best == i) return;
        head t = h[i]; h[i] = h[best]; h[best] = t;
        i = best;
    }
}

/* Step 1 of GSD and GER: X = the p near-equal blocks of the input, each sorted
 * by SR4 (payloads alongside); lo[k] = first index of block k, lo[p] = n. */
static int local_sort(const uint32_t* keys_in, const uint32_t* vals_in, size_t n, size_t p,
                      uint32_t* X, uint32_t* XV, uint64_t* lo)
{
    for (size_t k = 0; k <= p; ++k) lo[k] = (uint64_t)((k * (unsigned __int128)n) / p);
    for (size_t k = 0; k < p; ++k) {
        int rc = lsd_u32(keys_in + lo[k], vals_in ? vals_in + lo[k] : NULL, lo[k + 1] - lo[k],
                         8, 0, 32, X + lo[k], vals_in ? XV + lo[k] : NULL);
        if (rc) return rc;
    }
    return 0;
}

/* Steps 3-5 of GSD and GER, given the sample sorted by composite (Sk, Sg):
 * splitters, split by binary search, p-way merge into keys_out/vals_out. */
static int split_and_merge(const uint32_t* X, const uint32_t* XV, const uint64_t* lo, size_t n,
                           size_t p, size_t s, const uint32_t* Sk, const uint32_t* Sg,
                           uint32_t* keys_out, uint32_t* vals_out, uint64_t* cnt,
                           uint32_t* split_key, uint64_t* split_g)
{
    uint64_t* b = (uint64_t*)malloc(p * (p + 1) * sizeof(uint64_t));
    head* heap = (head*)malloc(p * sizeof(head));
    uint64_t* cur = (uint64_t*)malloc(p * sizeof(uint64_t));
    int rc = 0;
    const int has_vals = XV != NULL;
    if (!b || !heap || !cur) {
        rc = -2;
        goto done;
    }
    /* step 3: splitters = the (i s)-th smallest sample composites */
    for (size_t i = 1; i < p; ++i) {
        split_key[i - 1] = Sk[i * s - 1];
        split_g[i - 1] = Sg[i * s - 1];
    }

    /* step 4: split every sorted block around the splitters by binary search:
       b[k][i] = #{q in block k : (X[q], q) <= S_i}, b[k][0] = 0, b[k][p] = N_k */
    for (size_t k = 0; k < p; ++k) {
        uint64_t Nk = lo[k + 1] - lo[k];
        b[k * (p + 1) + 0] = 0;
        b[k * (p + 1) + p] = Nk;
        for (size_t i = 1; i < p; ++i) {
            uint64_t a = 0, e = Nk;                       /* first q with S_i < X_q */
            while (a < e) {
                uint64_t mid = a + (e - a) / 2;
                if (!comp_less(split_key[i - 1], split_g[i - 1], X[lo[k] + mid], lo[k] + mid))
                    a = mid + 1;
                else
                    e = mid;
            }
            b[k * (p + 1) + i] = a;
        }
        for (size_t j = 0; j < p; ++j)
            cnt[k * p + j] = b[k * (p + 1) + j + 1] - b[k * (p + 1) + j];
    }

    /* step 5: Y_j = p-way merge of X_{0,j} .. X_{p-1,j}; Y = Y_0 Y_1 ... */
    uint64_t o = 0;
    for (size_t j = 0; j < p; ++j) {
        size_t m = 0;
        for (size_t k = 0; k < p; ++k) {
            cur[k] = b[k * (p + 1) + j];
            if (cur[k] < b[k * (p + 1) + j + 1]) {
                heap[m].key = X[lo[k] + cur[k]];
                heap[m].run = (uint32_t)k;
                ++m;
            }
        }
        for (size_t i = m; i-- > 0;) heap_sift_down(heap, m, i);
        while (m) {
            uint32_t k = heap[0].run;
            if (o >= n) { rc = -3; goto done; }          /* runs overlap: split is broken */
            keys_out[o] = X[lo[k] + cur[k]];
            if (has_vals) vals_out[o] = XV[lo[k] + cur[k]];
            ++o;
            ++cur[k];
            if (cur[k] < b[(size_t)k * (p + 1) + j + 1]) {
                heap[0].key = X[lo[k] + cur[k]];
            } else {
                heap[0] = heap[--m];
            }
            if (m) heap_sift_down(heap, m, 0);
        }
    }
    if (o != n) rc = -3;

done:
    free(b); free(heap); free(cur);
    return rc;
}

int gsd_u32(const uint32_t* keys_in, const uint32_t* vals_in, size_t n,
            int p_req, int r,
            uint32_t* keys_out, uint32_t* vals_out,
            uint64_t* cnt /* p*p */, uint32_t* split_key /* p-1 */,
            uint64_t* split_g /* p-1 */, int* p_used)
{
    if (p_req < 1 || r < 1 || n == 0 || n >= ((uint64_t)1 << 32) ||
        !keys_in || !keys_out || (vals_in && !vals_out))
        return -1;
    size_t p = (size_t)p_req < n ? (size_t)p_req : n;
    *p_used = (int)p;
    const size_t s = (size_t)r * p;

    uint32_t* X = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* XV = vals_in ? (uint32_t*)malloc(n * sizeof(uint32_t)) : NULL;
    uint64_t* lo = (uint64_t*)malloc((p + 1) * sizeof(uint64_t));
    uint32_t* Tk = (uint32_t*)malloc(p * s * sizeof(uint32_t));
    uint32_t* Tg = (uint32_t*)malloc(p * s * sizeof(uint32_t));
    uint32_t* Sk = (uint32_t*)malloc(p * s * sizeof(uint32_t));
    uint32_t* Sg = (uint32_t*)malloc(p * s * sizeof(uint32_t));
    int rc = 0;
    if (!X || (vals_in && !XV) || !lo || !Tk || !Tg || !Sk || !Sg) {
        rc = -2;
        goto done;
    }
    /* step 1: local sorting of p near-equal blocks */
    rc = local_sort(keys_in, vals_in, n, p, X, XV, lo);
    if (rc) goto done;

    /* step 2: regular sample of s keys per block, the last one the block maximum */
    for (size_t k = 0; k < p; ++k) {
        uint64_t Nk = lo[k + 1] - lo[k];
        for (size_t j = 1; j <= s; ++j) {
            uint64_t q = (j * Nk + s - 1) / s - 1;          /* ceil(j Nk / s) - 1 */
            Tk[k * s + j - 1] = X[lo[k] + q];
            Tg[k * s + j - 1] = (uint32_t)(lo[k] + q);
        }
    }
    /* sort the sample by (key, g): T is laid out in block order, so g already
       increases along equal keys and a stable sort by key suffices */
    rc = lsd_u32(Tk, Tg, p * s, 8, 0, 32, Sk, Sg);
    if (rc) goto done;

    /* steps 3-5 */
    rc = split_and_merge(X, XV, lo, n, p, s, Sk, Sg, keys_out, vals_out, cnt, split_key, split_g);

done:
    free(X); free(XV); free(lo); free(Tk); free(Tg); free(Sk); free(Sg);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* GER, Algorithm 2 (Section 3.3): the GSD skeleton with a random sample.
 *
 * Readings where the paper is silent:
 *  - Steps 1 and 3-5 as in GSD above (same blocks, composites, split and
 *    stable merge).
 *  - Step 2 draws s p - 1 keys "uniformly at random from the keys of all X_k"
 *    with replacement: the draws are the caller's positions pos[0 .. s p - 1)
 *    into X, each in [0, n), so that a test and the GPU use the same draws.
 *    Sample element i is the composite (X[pos[i]], pos[i]).
 *  - The sample is sorted by composite (SR4 by position, then SR4 by key,
 *    both stable) instead of BTN; splitter i is the (i s)-th smallest.
 */
int ger_u32(const uint32_t* keys_in, const uint32_t* vals_in, size_t n, int p_req, int s_req,
            const uint32_t* pos, size_t npos, uint32_t* keys_out, uint32_t* vals_out,
            uint64_t* cnt /* p*p */, uint32_t* split_key /* p-1 */,
            uint64_t* split_g /* p-1 */, int* p_used)
{
    if (p_req < 1 || s_req < 1 || n == 0 || n >= ((uint64_t)1 << 32) ||
        !keys_in || !keys_out || (vals_in && !vals_out))
        return -1;
    size_t p = (size_t)p_req < n ? (size_t)p_req : n;
    *p_used = (int)p;
    const size_t s = (size_t)s_req;
    const size_t m = s * p - 1;            /* sample size */
    if (npos < m || (m && !pos)) return -1;
    for (size_t i = 0; i < m; ++i)
        if (pos[i] >= n) return -1;

    uint32_t* X = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* XV = vals_in ? (uint32_t*)malloc(n * sizeof(uint32_t)) : NULL;
    uint64_t* lo = (uint64_t*)malloc((p + 1) * sizeof(uint64_t));
    uint32_t* Tk = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* Tg = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* Uk = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* Ug = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    int rc = 0;
    if (!X || (vals_in && !XV) || !lo || !Tk || !Tg || !Uk || !Ug) {
        rc = -2;
        goto done;
    }
    /* step 1 */
    rc = local_sort(keys_in, vals_in, n, p, X, XV, lo);
    if (rc) goto done;
    /* step 2: the random sample, sorted by (key, position) */
    for (size_t i = 0; i < m; ++i) {
        Tg[i] = pos[i];
        Tk[i] = X[pos[i]];
    }
    rc = lsd_u32(Tg, Tk, m, 8, 0, 32, Ug, Uk);        /* by position */
    if (rc) goto done;
    rc = lsd_u32(Uk, Ug, m, 8, 0, 32, Tk, Tg);        /* then by key, stably */
    if (rc) goto done;
    /* steps 3-5 */
    rc = split_and_merge(X, XV, lo, n, p, s, Tk, Tg, keys_out, vals_out, cnt, split_key, split_g);

done:
    free(X); free(XV); free(lo); free(Tk); free(Tg); free(Uk); free(Ug);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* GVR, Algorithm 3 (Section 3.3): sample first, split the unsorted blocks,
 * sort each bucket.
 *
 * Readings where the paper is silent:
 *  - Blocks X_k = [floor(k n / p), floor((k+1) n / p)) of the input, p clamped
 *    to n.
 *  - Step 1 draws s p - 1 keys uniformly at random, with replacement, from the
 *    input: the draws are the caller's input positions pos[0 .. s p - 1).
 *    Sample element i is the composite (x[pos[i]], pos[i]); the sample is
 *    sorted by composite (SR4 by position, then SR4 by key) instead of BTN.
 *  - Step 2: splitter i is the (i s)-th smallest sample composite.
 *  - Step 3: an element e = (x_q, q) of block k belongs to X_{k,j} with
 *    j = #{i : S_i < e} (binary search over the splitters); X_{k,j} keeps input
 *    order (a stable count sort by j).
 *  - Step 4: Y_j = X_{0,j} ... X_{p-1,j} is sorted by SR4 (stable), so equal
 *    keys stay in input order and the result is the stable sort.
 */
int gvr_u32(const uint32_t* keys_in, const uint32_t* vals_in, size_t n, int p_req, int s_req,
            const uint32_t* pos, size_t npos, uint32_t* keys_out, uint32_t* vals_out,
            uint64_t* cnt /* p*p */, uint32_t* split_key /* p-1 */,
            uint64_t* split_g /* p-1 */, int* p_used)
{
    if (p_req < 1 || s_req < 1 || n == 0 || n >= ((uint64_t)1 << 32) ||
        !keys_in || !keys_out || (vals_in && !vals_out))
        return -1;
    size_t p = (size_t)p_req < n ? (size_t)p_req : n;
    *p_used = (int)p;
    const size_t s = (size_t)s_req;
    const size_t m = s * p - 1;
    if (npos < m || (m && !pos)) return -1;
    for (size_t i = 0; i < m; ++i)
        if (pos[i] >= n) return -1;

    uint32_t* Tk = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* Tg = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* Uk = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* Ug = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* bucket = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint64_t* start = (uint64_t*)malloc((p + 1) * sizeof(uint64_t));
    uint32_t* Y = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* YV = vals_in ? (uint32_t*)malloc(n * sizeof(uint32_t)) : NULL;
    int rc = 0;
    if (!Tk || !Tg || !Uk || !Ug || !bucket || !start || !Y || (vals_in && !YV)) {
        rc = -2;
        goto done;
    }
    /* step 1: the random sample, sorted by (key, position) */
    for (size_t i = 0; i < m; ++i) {
        Tg[i] = pos[i];
        Tk[i] = keys_in[pos[i]];
    }
    rc = lsd_u32(Tg, Tk, m, 8, 0, 32, Ug, Uk);        /* by input position */
    if (rc) goto done;
    rc = lsd_u32(Uk, Ug, m, 8, 0, 32, Tk, Tg);        /* then by key, stably */
    if (rc) goto done;
    /* step 2: splitters */
    for (size_t i = 1; i < p; ++i) {
        split_key[i - 1] = Tk[i * s - 1];
        split_g[i - 1] = Tg[i * s - 1];
    }
    /* step 3: bucket of every element = number of splitters below it */
    memset(cnt, 0, p * p * sizeof(uint64_t));
    for (size_t q = 0; q < n; ++q) {
        size_t a = 0, e = p - 1;                      /* first splitter not below x_q */
        while (a < e) {
            size_t mid = a + (e - a) / 2;
            if (comp_less(split_key[mid], split_g[mid], keys_in[q], q))
                a = mid + 1;
            else
                e = mid;
        }
        bucket[q] = (uint32_t)a;
        size_t k = (size_t)(((unsigned __int128)q * p + p - 1) / n);   /* q's block */
        while (k > 0 && (uint64_t)((k * (unsigned __int128)n) / p) > q) --k;
        while ((uint64_t)(((k + 1) * (unsigned __int128)n) / p) <= q) ++k;
        cnt[k * p + a] += 1;
    }
    /* route: Y_j = the elements of bucket j in input order (stable count sort) */
    memset(start, 0, (p + 1) * sizeof(uint64_t));
    for (size_t q = 0; q < n; ++q) start[bucket[q] + 1] += 1;
    for (size_t j = 0; j < p; ++j) start[j + 1] += start[j];
    for (size_t q = 0; q < n; ++q) {
        uint64_t o = start[bucket[q]]++;
        Y[o] = keys_in[q];
        if (vals_in) YV[o] = vals_in[q];
    }
    /* step 4: every bucket sorted by SR4; start[j] is now the end of bucket j */
    for (size_t j = 0; j < p; ++j) {
        uint64_t lo = j ? start[j - 1] : 0, hi = start[j];
        rc = lsd_u32(Y + lo, vals_in ? YV + lo : NULL, hi - lo, 8, 0, 32, keys_out + lo,
                     vals_in ? vals_out + lo : NULL);
        if (rc) goto done;
    }

done:
    free(Tk); free(Tg); free(Uk); free(Ug); free(bucket); free(start); free(Y); free(YV);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Signed and floating-point keys (not in the paper, which sorts unsigned
 * integers): a stable merge sort by comparison.
 *   kind 1  two's complement integers, ordered as signed numbers;
 *   kind 2  IEEE 754 bit patterns ordered by totalOrder: every key with the
 *           sign bit set precedes every key without it; among keys without
 *           it a larger bit pattern is larger, among keys with it a larger
 *           bit pattern is smaller (-NaN < -inf < ... < -0 < +0 < ... < +inf
 *           < +NaN).
 * Ties keep input order, so with payloads the result is the stable sort.   */
static int cmp_kind(uint64_t a, uint64_t b, int bits, int kind)
{
    const uint64_t sign = (uint64_t)1 << (bits - 1);
    const int sa = (a & sign) != 0, sb = (b & sign) != 0;
    if (sa != sb) return sa ? -1 : 1;                 /* negative first */
    if (a == b) return 0;
    if (kind == 1) return a < b ? -1 : 1;             /* same sign: bits order as numbers */
    if (!sa) return a < b ? -1 : 1;                   /* float, both positive */
    return a < b ? 1 : -1;                            /* float, both negative: reversed */
}

static int merge_sort_kind(uint64_t* k, uint32_t* v, size_t n, int bits, int kind)
{
    uint64_t* tk = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint32_t* tv = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!tk || !tv) {
        free(tk); free(tv);
        return -2;
    }
    for (size_t width = 1; width < n; width *= 2) {
        for (size_t lo = 0; lo < n; lo += 2 * width) {
            size_t mid = lo + width < n ? lo + width : n;
            size_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            size_t i = lo, j = mid, o = lo;
            while (i < mid && j < hi) {                   /* left first on ties: stable */
                if (cmp_kind(k[j], k[i], bits, kind) < 0) { tk[o] = k[j]; tv[o++] = v[j++]; }
                else { tk[o] = k[i]; tv[o++] = v[i++]; }
            }
            while (i < mid) { tk[o] = k[i]; tv[o++] = v[i++]; }
            while (j < hi) { tk[o] = k[j]; tv[o++] = v[j++]; }
        }
        memcpy(k, tk, n * sizeof(uint64_t));
        memcpy(v, tv, n * sizeof(uint32_t));
    }
    free(tk);
    free(tv);
    return 0;
}

/* keys: n keys of `bits` (32 or 64) bits in 64-bit slots; vals may be NULL. */
int sort_kind(uint64_t* keys, uint32_t* vals, size_t n, int bits, int kind)
{
    if ((bits != 32 && bits != 64) || (kind != 1 && kind != 2) || (n && !keys)) return -1;
    uint32_t* v = vals ? vals : (uint32_t*)calloc(n ? n : 1, sizeof(uint32_t));
    if (!v) return -2;
    int rc = merge_sort_kind(keys, v, n, bits, kind);
    if (!vals) free(v);
    return rc;
}
