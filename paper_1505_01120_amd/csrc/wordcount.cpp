// WordCount (sec. 3.2.3): words of a device-resident byte stream counted under
// their 64-bit FNV-1a key, in per-block LDS tables whose misses go to
// per-partition spill regions; a merge pass counts each partition's spilled
// keys and adds them to one global open-addressing table, which is then
// compacted into the caller's arrays.
#include <algorithm>
#include <cstring>
#include <string>

#include "runtime.h"

using namespace sparkcl;

extern "C" {

int sparkcl_wordcount(sparkcl_ctx *ctx, const uint8_t *text, uint64_t nbytes, uint64_t *keys,
                      uint64_t *counts, uint64_t capacity, uint64_t *ndistinct,
                      uint64_t *nwords, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if (!ndistinct || !nwords || (nbytes && !text) || (capacity && (!keys || !counts)))
        return fail(SPARKCL_EINVAL, "NULL argument");
    *ndistinct = 0;
    *nwords = 0;
    if (nbytes == 0)
        return SPARKCL_OK;
    if (nbytes > kMaxN)
        return fail(SPARKCL_ETOOBIG, "text of " + std::to_string(nbytes) +
                                         " bytes exceeds 2^40");
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // open addressing at load <= 1/2: room for capacity + 1 keys (so one key
    // past the capacity is still seen), never more than the text can hold
    uint64_t need = std::min<uint64_t>(capacity + 1, nbytes / 2 + 1);
    uint64_t slots = 1024;
    while (slots < 2 * need)
        slots *= 2;
    if (!ctx->occ_wordcount) {
        int occ = 0;
        if (wordcount_blocks_per_cu(&occ) != SPARKCL_OK || occ < 1)
            occ = 1;
        ctx->occ_wordcount = occ;
    }
    const uint64_t nchunks = (nbytes + 4095) / 4096;
    const uint32_t grid =
        (uint32_t)std::min<uint64_t>(nchunks, (uint64_t)ctx->occ_wordcount * ctx->cus);
    const uint64_t table_bytes = slots * 16 + 64;
    // Spill regions: room for one spilled word per 16 bytes of each scan
    // block's share of the text (a quarter more for the spread between
    // partitions); words past a full region go to the table directly.  Left
    // out when the arena cannot hold them.
    const uint64_t parts = 1ull << kWcPartBits;
    uint64_t cap = nbytes / ((uint64_t)grid * parts * 16);
    cap = cap + cap / 4 + 16;
    const uint64_t spill_bytes = (uint64_t)grid * parts * (cap * 8 + 4);
    uint64_t bytes = table_bytes + spill_bytes;
    uint64_t off = ctx->arena.alloc(bytes);
    if (off == Arena::kFail) {
        cap = 0;
        bytes = table_bytes;
        off = ctx->arena.alloc(bytes);
    }
    if (off == Arena::kFail)
        return fail(SPARKCL_ENOMEM, "word-count table of " + std::to_string(bytes) +
                                        " bytes does not fit the arena");
    char *base = static_cast<char *>(ctx->dev(off));
    WcArgs a{};
    a.text = text;
    a.n = nbytes;
    a.keys = reinterpret_cast<uint64_t *>(base);
    a.counts = reinterpret_cast<uint64_t *>(base + slots * 8);
    a.ctl = reinterpret_cast<uint64_t *>(base + slots * 16);
    a.mask = slots - 1;
    a.spill_cap = (uint32_t)cap;
    if (cap) {
        a.spill = reinterpret_cast<uint64_t *>(base + table_bytes);
        a.spill_cnt = reinterpret_cast<uint32_t *>(base + table_bytes +
                                                   (uint64_t)grid * parts * cap * 8);
    }
    // merge: eight blocks per partition (each merge block's loads are a
    // few hundred bytes per region, so it takes many blocks to keep enough
    // of them in flight), at least one per CU in all
    const uint32_t per_part = (uint32_t)std::max<uint64_t>(8, (uint64_t)ctx->cus / parts);
    const uint32_t cgrid =
        (uint32_t)std::min<uint64_t>((slots + kBlock - 1) / kBlock, 4ull * ctx->cus);
    // (only the table and the counters need clearing: every spill slot read
    // by the merge was written by the scan)
    if ((rc = ensure_pinned(ctx, 1)) == SPARKCL_OK &&
        (rc = launch_zero(base, table_bytes, s)) == SPARKCL_OK &&
        (rc = launch_wordcount(a, grid, s)) == SPARKCL_OK &&
        (!cap || (rc = launch_wc_merge(a, grid, per_part, s)) == SPARKCL_OK) &&
        (rc = launch_wc_compact(a, keys, counts, capacity, cgrid, s)) == SPARKCL_OK) {
        hipError_t e = hipMemcpyAsync(ctx->pinned, a.ctl, 32, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            rc = fail_hip(e, "word count");
    } else if (rc != SPARKCL_OK) {
        (void)hipStreamSynchronize(s);
        rc = fail(rc, "word-count launch failed");
    }
    ctx->arena.release(off);
    if (rc != SPARKCL_OK)
        return rc;
    uint64_t ctl[4];
    std::memcpy(ctl, ctx->pinned, sizeof(ctl));
    *nwords = ctl[0];
    *ndistinct = ctl[3];
    if (ctl[2] || ctl[3] > capacity)
        return fail(SPARKCL_ETOOBIG, "more distinct words than the capacity of " +
                                         std::to_string(capacity));
    return SPARKCL_OK;
}

int sparkcl_wordcount_locate(sparkcl_ctx *ctx, const uint8_t *text, uint64_t nbytes,
                             const uint64_t *keys, uint64_t nkeys, uint64_t *offsets,
                             void *stream)
{
    int rc = check_ctx(ctx);
    if (rc != SPARKCL_OK)
        return rc;
    if ((nbytes && !text) || (nkeys && (!keys || !offsets)))
        return fail(SPARKCL_EINVAL, "NULL argument");
    if (nkeys == 0)
        return SPARKCL_OK;
    if (nbytes > kMaxN)
        return fail(SPARKCL_ETOOBIG, "text of " + std::to_string(nbytes) +
                                         " bytes exceeds 2^40");
    if (nkeys > 0xFFFFFFFFull)
        return fail(SPARKCL_ETOOBIG, "more than 2^32 - 1 keys");
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t slots = 1024;
    while (slots < 2 * nkeys)
        slots *= 2;
    if (!ctx->occ_wordcount) {
        int occ = 0;
        if (wordcount_blocks_per_cu(&occ) != SPARKCL_OK || occ < 1)
            occ = 1;
        ctx->occ_wordcount = occ;
    }
    const uint64_t nchunks = std::max<uint64_t>(1, (nbytes + 4095) / 4096);
    const uint32_t grid =
        (uint32_t)std::min<uint64_t>(nchunks, (uint64_t)ctx->occ_wordcount * ctx->cus);
    // table keys, then control words, then the key indices
    const uint64_t zero_bytes = slots * 8 + 64;
    const uint64_t bytes = zero_bytes + slots * 4;
    const uint64_t off = ctx->arena.alloc(bytes);
    if (off == Arena::kFail)
        return fail(SPARKCL_ENOMEM, "word lookup table of " + std::to_string(bytes) +
                                        " bytes does not fit the arena");
    char *base = static_cast<char *>(ctx->dev(off));
    WlArgs l{};
    l.text = text;
    l.n = nbytes;
    l.keys = keys;
    l.nkeys = nkeys;
    l.offsets = offsets;
    l.tkeys = reinterpret_cast<uint64_t *>(base);
    l.ctl = reinterpret_cast<uint64_t *>(base + slots * 8);
    l.tidx = reinterpret_cast<uint32_t *>(base + zero_bytes);
    l.mask = slots - 1;
    if ((rc = ensure_pinned(ctx, 1)) == SPARKCL_OK &&
        (rc = launch_zero(base, zero_bytes, s)) == SPARKCL_OK &&
        (rc = launch_wordcount_locate(l, grid, s)) == SPARKCL_OK) {
        hipError_t e = hipMemcpyAsync(ctx->pinned, l.ctl, 16, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            rc = fail_hip(e, "word locate");
    } else if (rc != SPARKCL_OK) {
        (void)hipStreamSynchronize(s);
        rc = fail(rc, "word-locate launch failed");
    }
    ctx->arena.release(off);
    if (rc != SPARKCL_OK)
        return rc;
    uint64_t ctl[2];
    std::memcpy(ctl, ctx->pinned, sizeof(ctl));
    if (ctl[1])
        return fail(SPARKCL_EINVAL, "a key appears twice in keys");
    return SPARKCL_OK;
}

} // extern "C"
