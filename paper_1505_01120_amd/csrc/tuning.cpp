// Tile-size table: defaults, validation and the JSON cache (see tuning.h).
#include "tuning.h"

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

namespace sparkcl {

namespace {

const char *kModeNames[SPARKCL_TUNE_MODES] = {"per_launch", "batched", "serve"};
const char *kKernelNames[3] = {"poly", "fmul", "mc_pi"};

uint32_t clamp_log2(int v)
{
    if (v < (int)kMinTileLog2)
        v = (int)kMinTileLog2;
    if (v > (int)kMaxTileLog2)
        v = (int)kMaxTileLog2;
    return 1u << v;
}

// ---- a small JSON reader for the cache format (objects, arrays, strings,
// non-negative integers) -----------------------------------------------------
struct Json {
    enum Kind { NUL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    std::string str;
    std::vector<Json> arr;
    std::vector<std::pair<std::string, Json>> obj;
    const Json *get(const char *k) const
    {
        for (auto &kv : obj)
            if (kv.first == k)
                return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const std::string &s;
    size_t i = 0;
    std::string err;
    explicit Parser(const std::string &text) : s(text) {}
    void ws()
    {
        while (i < s.size() && std::isspace((unsigned char)s[i]))
            ++i;
    }
    bool fail(const char *m)
    {
        if (err.empty())
            err = std::string(m) + " at offset " + std::to_string(i);
        return false;
    }
    bool str(std::string *out)
    {
        if (i >= s.size() || s[i] != '"')
            return fail("expected string");
        ++i;
        out->clear();
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\') {
                ++i;
                if (i >= s.size())
                    return fail("bad escape");
            }
            out->push_back(s[i++]);
        }
        if (i >= s.size())
            return fail("unterminated string");
        ++i;
        return true;
    }
    bool value(Json *v, int depth)
    {
        if (depth > 16)
            return fail("nesting too deep");
        ws();
        if (i >= s.size())
            return fail("unexpected end");
        char c = s[i];
        if (c == '{') {
            v->kind = Json::OBJ;
            ++i;
            ws();
            if (i < s.size() && s[i] == '}') {
                ++i;
                return true;
            }
            for (;;) {
                ws();
                std::string k;
                if (!str(&k))
                    return false;
                ws();
                if (i >= s.size() || s[i] != ':')
                    return fail("expected ':'");
                ++i;
                Json child;
                if (!value(&child, depth + 1))
                    return false;
                v->obj.emplace_back(k, std::move(child));
                ws();
                if (i < s.size() && s[i] == ',') {
                    ++i;
                    continue;
                }
                if (i < s.size() && s[i] == '}') {
                    ++i;
                    return true;
                }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            v->kind = Json::ARR;
            ++i;
            ws();
            if (i < s.size() && s[i] == ']') {
                ++i;
                return true;
            }
            for (;;) {
                Json child;
                if (!value(&child, depth + 1))
                    return false;
                v->arr.push_back(std::move(child));
                ws();
                if (i < s.size() && s[i] == ',') {
                    ++i;
                    continue;
                }
                if (i < s.size() && s[i] == ']') {
                    ++i;
                    return true;
                }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v->kind = Json::STR;
            return str(&v->str);
        }
        if (std::isdigit((unsigned char)c) || c == '-') {
            size_t j = i;
            if (s[j] == '-')
                ++j;
            while (j < s.size() && (std::isdigit((unsigned char)s[j]) || s[j] == '.' ||
                                    s[j] == 'e' || s[j] == 'E' || s[j] == '+' || s[j] == '-'))
                ++j;
            v->kind = Json::NUM;
            v->num = std::strtod(s.c_str() + i, nullptr);
            i = j;
            return true;
        }
        if (s.compare(i, 4, "null") == 0) {
            i += 4;
            v->kind = Json::NUL;
            return true;
        }
        return fail("unexpected character");
    }
};

} // namespace

void tuning_defaults(sparkcl_tuning *t)
{
    std::memset(t, 0, sizeof(*t));
    for (int k = 0; k < 3; ++k) {
        t->block[k] = 256;
        t->unroll[k] = 4;
    }
    t->block_many = 256;
    // blocks_per_cu 0: as many as fit (occupancy)
    for (uint32_t b = 0; b < SPARKCL_TUNE_BUCKETS; ++b) {
        // One launch per partition: aim at ~2048 tiles so the grid fills the
        // chip, without going below 4K elements per 256-thread block.
        t->tile[TM_PER_LAUNCH][0][b] = clamp_log2(std::min<int>((int)b - 11, 16));
        t->tile[TM_PER_LAUNCH][1][b] = clamp_log2(std::min<int>((int)b - 11, 16));
        t->tile[TM_PER_LAUNCH][2][b] = clamp_log2(std::min<int>((int)b - 11, 18));
        if (t->tile[TM_PER_LAUNCH][0][b] < 4096u)
            t->tile[TM_PER_LAUNCH][0][b] = t->tile[TM_PER_LAUNCH][1][b] = 4096u;
        if (t->tile[TM_PER_LAUNCH][2][b] < 4096u)
            t->tile[TM_PER_LAUNCH][2][b] = 4096u;
        // Many partitions in one persistent launch: bigger tiles, fewer
        // queue operations; small partitions stay one tile.
        t->tile[TM_BATCHED][0][b] = clamp_log2(std::min<int>((int)b, 15));
        t->tile[TM_BATCHED][1][b] = clamp_log2(std::min<int>((int)b, 15));
        t->tile[TM_BATCHED][2][b] = clamp_log2(std::min<int>((int)b, 16));
        // Serving: latency first, a task spreads over many blocks.
        t->tile[TM_SERVE][0][b] = clamp_log2(std::min<int>((int)b - 4, 14));
        t->tile[TM_SERVE][1][b] = clamp_log2(std::min<int>((int)b - 4, 14));
        t->tile[TM_SERVE][2][b] = clamp_log2(std::min<int>((int)b - 4, 14));
    }
}

int tuning_validate(const sparkcl_tuning *t, std::string *why)
{
    if (!t) {
        if (why)
            *why = "null tuning table";
        return SPARKCL_EINVAL;
    }
    if (t->blocks_per_cu_mc_only > 32) {
        if (why)
            *why = "blocks_per_cu_mc_only above 32";
        return SPARKCL_EINVAL;
    }
    if (t->blocks_per_cu_many > 32) {
        if (why)
            *why = "blocks_per_cu_many above 32";
        return SPARKCL_EINVAL;
    }
    for (int k = 0; k < 3; ++k)
        if (t->blocks_per_cu[k] > 32) {
            if (why)
                *why = "blocks_per_cu above 32";
            return SPARKCL_EINVAL;
        }
    auto block_ok = [](uint32_t b) { return b == 0 || b == 256 || b == 512 || b == 1024; };
    auto unroll_ok = [](uint32_t u) { return u == 0 || u == 2 || u == 4 || u == 8; };
    for (int k = 0; k < 3; ++k)
        if (!block_ok(t->block[k]) || !unroll_ok(t->unroll[k])) {
            if (why)
                *why = std::string("block[") + kKernelNames[k] + "] = " +
                       std::to_string(t->block[k]) + " or unroll = " +
                       std::to_string(t->unroll[k]) +
                       " not in {0, 256, 512, 1024} / {0, 2, 4, 8}";
            return SPARKCL_EINVAL;
        }
    if (!block_ok(t->block_many)) {
        if (why)
            *why = "block_many = " + std::to_string(t->block_many) +
                   " not in {0, 256, 512, 1024}";
        return SPARKCL_EINVAL;
    }
    for (int k = 0; k < 2; ++k)
        if (t->many_tiles_per_cu[k] > 4096) {
            if (why)
                *why = "many_tiles_per_cu[" + std::to_string(k) + "] = " +
                       std::to_string(t->many_tiles_per_cu[k]) + " is above 4096";
            return SPARKCL_EINVAL;
        }
    for (int k = 0; k < 3; ++k) {
        const uint32_t v = t->tile_many[k];
        if (v != 0 && (v < (1u << kMinTileLog2) || v > (1u << kMaxTileLog2) || (v & (v - 1)))) {
            if (why)
                *why = std::string("tile_many[") + kKernelNames[k] + "] = " +
                       std::to_string(v) + " is neither 0 nor a power of two in [2^10, 2^22]";
            return SPARKCL_EINVAL;
        }
    }
    for (int m = 0; m < SPARKCL_TUNE_MODES; ++m)
        for (int k = 0; k < 3; ++k)
            for (int b = 0; b < SPARKCL_TUNE_BUCKETS; ++b) {
                const uint32_t v = t->tile[m][k][b];
                if (v < (1u << kMinTileLog2) || v > (1u << kMaxTileLog2) || (v & (v - 1))) {
                    if (why)
                        *why = std::string("tile[") + kModeNames[m] + "][" +
                               kKernelNames[k] + "][" + std::to_string(b) +
                               "] = " + std::to_string(v) +
                               " is not a power of two in [2^10, 2^22]";
                    return SPARKCL_EINVAL;
                }
            }
    return SPARKCL_OK;
}

uint32_t tile_for(const sparkcl_tuning &t, int mode, uint32_t kid, uint64_t n)
{
    return t.tile[mode][kid - 1][size_bucket(n)];
}

bool tuning_parse_json(const std::string &text,
                       std::map<std::string, sparkcl_tuning> *out, std::string *err)
{
    Parser p(text);
    Json root;
    if (!p.value(&root, 0)) {
        if (err)
            *err = p.err;
        return false;
    }
    if (root.kind != Json::OBJ) {
        if (err)
            *err = "top level is not an object";
        return false;
    }
    for (auto &arch : root.obj) {
        sparkcl_tuning t;
        tuning_defaults(&t);
        const Json &e = arch.second;
        if (e.kind != Json::OBJ) {
            if (err)
                *err = "entry for " + arch.first + " is not an object";
            return false;
        }
        if (const Json *b = e.get("blocks_per_cu")) {
            if (b->kind == Json::NUM) {
                for (int k = 0; k < 3; ++k)
                    t.blocks_per_cu[k] = (uint32_t)b->num;
            } else if (b->kind == Json::ARR && b->arr.size() == 3) {
                for (int k = 0; k < 3; ++k)
                    t.blocks_per_cu[k] = (uint32_t)b->arr[k].num;
            } else {
                if (err)
                    *err = "blocks_per_cu must be a number or an array of 3";
                return false;
            }
        }
        if (const Json *b = e.get("blocks_per_cu_many"))
            t.blocks_per_cu_many = (uint32_t)b->num;
        if (const Json *b = e.get("blocks_per_cu_mc_only"))
            t.blocks_per_cu_mc_only = (uint32_t)b->num;
        for (const char *name : {"block", "unroll"}) {
            const Json *b = e.get(name);
            if (!b)
                continue;
            if (b->kind != Json::ARR || b->arr.size() != 3) {
                if (err)
                    *err = std::string(name) + " must be an array of 3";
                return false;
            }
            for (int k = 0; k < 3; ++k)
                (name[0] == 'b' ? t.block : t.unroll)[k] = (uint32_t)b->arr[k].num;
        }
        if (const Json *b = e.get("block_many"))
            t.block_many = (uint32_t)b->num;
        if (const Json *b = e.get("many_tiles_per_cu")) {
            if (b->kind != Json::ARR || b->arr.size() != 2) {
                if (err)
                    *err = "many_tiles_per_cu must be an array of 2";
                return false;
            }
            for (int k = 0; k < 2; ++k)
                t.many_tiles_per_cu[k] = (uint32_t)b->arr[k].num;
        }
        if (const Json *b = e.get("tile_many")) {
            if (b->kind != Json::ARR || b->arr.size() != 3) {
                if (err)
                    *err = "tile_many must be an array of 3";
                return false;
            }
            for (int k = 0; k < 3; ++k)
                t.tile_many[k] = (uint32_t)b->arr[k].num;
        }
        if (const Json *tile = e.get("tile")) {
            for (int m = 0; m < SPARKCL_TUNE_MODES; ++m) {
                const Json *mj = tile->get(kModeNames[m]);
                if (!mj)
                    continue;
                for (int k = 0; k < 3; ++k) {
                    const Json *kj = mj->get(kKernelNames[k]);
                    if (!kj)
                        continue;
                    if (kj->kind != Json::ARR || kj->arr.size() != SPARKCL_TUNE_BUCKETS) {
                        if (err)
                            *err = std::string("tile.") + kModeNames[m] + "." +
                                   kKernelNames[k] + " must be an array of 32 sizes";
                        return false;
                    }
                    for (int b = 0; b < SPARKCL_TUNE_BUCKETS; ++b)
                        t.tile[m][k][b] = (uint32_t)kj->arr[b].num;
                }
            }
        }
        std::string why;
        if (tuning_validate(&t, &why) != SPARKCL_OK) {
            if (err)
                *err = arch.first + ": " + why;
            return false;
        }
        (*out)[arch.first] = t;
    }
    return true;
}

std::string tuning_to_json(const std::map<std::string, sparkcl_tuning> &all)
{
    std::ostringstream o;
    o << "{\n";
    size_t ai = 0;
    for (auto &kv : all) {
        const sparkcl_tuning &t = kv.second;
        o << " \"" << kv.first << "\": {\n  \"blocks_per_cu\": [" << t.blocks_per_cu[0]
          << ", " << t.blocks_per_cu[1] << ", " << t.blocks_per_cu[2]
          << "],\n  \"blocks_per_cu_many\": " << t.blocks_per_cu_many
          << ",\n  \"blocks_per_cu_mc_only\": " << t.blocks_per_cu_mc_only
          << ",\n  \"tile_many\": [" << t.tile_many[0] << ", " << t.tile_many[1] << ", "
          << t.tile_many[2] << "],\n  \"block\": [" << t.block[0] << ", " << t.block[1] << ", "
          << t.block[2] << "],\n  \"block_many\": " << t.block_many << ",\n  \"unroll\": ["
          << t.unroll[0] << ", " << t.unroll[1] << ", " << t.unroll[2]
          << "],\n  \"many_tiles_per_cu\": [" << t.many_tiles_per_cu[0] << ", "
          << t.many_tiles_per_cu[1] << "],\n  \"tile\": {\n";
        for (int m = 0; m < SPARKCL_TUNE_MODES; ++m) {
            o << "   \"" << kModeNames[m] << "\": {\n";
            for (int k = 0; k < 3; ++k) {
                o << "    \"" << kKernelNames[k] << "\": [";
                for (int b = 0; b < SPARKCL_TUNE_BUCKETS; ++b)
                    o << t.tile[m][k][b] << (b + 1 < SPARKCL_TUNE_BUCKETS ? ", " : "");
                o << "]" << (k < 2 ? "," : "") << "\n";
            }
            o << "   }" << (m + 1 < SPARKCL_TUNE_MODES ? "," : "") << "\n";
        }
        o << "  }\n }" << (++ai < all.size() ? "," : "") << "\n";
    }
    o << "}\n";
    return o.str();
}

bool tuning_load_file(const std::string &path, const std::string &arch,
                      sparkcl_tuning *out, std::string *err)
{
    std::ifstream f(path);
    if (!f) {
        if (err)
            *err = "cannot open " + path;
        return false;
    }
    std::stringstream ss;
    ss << f.rdbuf();
    std::map<std::string, sparkcl_tuning> all;
    if (!tuning_parse_json(ss.str(), &all, err))
        return false;
    auto it = all.find(arch);
    if (it == all.end()) {
        if (err)
            *err = "no entry for " + arch + " in " + path;
        return false;
    }
    *out = it->second;
    return true;
}

bool tuning_save_file(const std::string &path, const std::string &arch,
                      const sparkcl_tuning &t, std::string *err)
{
    std::map<std::string, sparkcl_tuning> all;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            std::string ignore;
            tuning_parse_json(ss.str(), &all, &ignore); // keep what parses
        }
    }
    all[arch] = t;
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) {
            if (err)
                *err = "cannot write " + tmp;
            return false;
        }
        f << tuning_to_json(all);
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        if (err)
            *err = "cannot rename " + tmp + " to " + path;
        return false;
    }
    return true;
}

} // namespace sparkcl
