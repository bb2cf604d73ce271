// On-disk cache of packed fast-form plans (see plan_cache.h).
#include "plan_cache.h"

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <type_traits>
#include <unistd.h>
#include <vector>

namespace sht {
namespace idbf {

namespace {

constexpr char kMagic[8] = {'S', 'H', 'T', 'P', 'L', 'A', 'N', 0};
constexpr uint32_t kFormat = 1;
// bump when the builder or the packer changes what a plan contains
constexpr int kPlanVersion = 3;

uint64_t fnv1a(const unsigned char *p, size_t n) {
    uint64_t h = 1469598103934665603ULL;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}

struct Writer {
    std::vector<unsigned char> b;
    template <typename T> void pod(const T &v) {
        static_assert(std::is_trivially_copyable<T>::value, "pod");
        const unsigned char *p = reinterpret_cast<const unsigned char *>(&v);
        b.insert(b.end(), p, p + sizeof(T));
    }
    template <typename T> void vec(const std::vector<T> &v) {
        static_assert(std::is_trivially_copyable<T>::value, "pod");
        pod<uint64_t>(v.size());
        const unsigned char *p = reinterpret_cast<const unsigned char *>(v.data());
        b.insert(b.end(), p, p + v.size() * sizeof(T));
    }
};

struct Reader {
    const unsigned char *p;
    size_t n, at = 0;
    bool ok = true;
    template <typename T> void pod(T &v) {
        if (!ok || n - at < sizeof(T)) {
            ok = false;
            return;
        }
        std::memcpy(&v, p + at, sizeof(T));
        at += sizeof(T);
    }
    template <typename T> void vec(std::vector<T> &v) {
        uint64_t k = 0;
        pod(k);
        if (!ok || k > (n - at) / sizeof(T)) {
            ok = false;
            return;
        }
        v.resize(k);
        std::memcpy(v.data(), p + at, k * sizeof(T));
        at += k * sizeof(T);
    }
};

void put_program(Writer &w, const Program &p) {
    w.vec(p.ops);
    w.vec(p.op_task);
    w.vec(p.subs);
    w.vec(p.idx);
    w.vec(p.vals);
    w.vec(p.stages);
    w.pod(p.n_work_stages);
    w.pod(p.scr_rows);
    w.pod(p.in_rows);
    w.pod(p.out_rows);
    w.pod(p.max_n_out);
    w.pod(p.max_n_in);
    w.vec(p.fgroups);
    w.vec(p.flevels);
    w.vec(p.fops);
    w.vec(p.fsubs);
    w.pod(p.f_max_lds_rows);
    w.pod(p.fused_ok);
    w.pod(p.f_extra_rows);
}

void get_program(Reader &r, Program &p) {
    r.vec(p.ops);
    r.vec(p.op_task);
    r.vec(p.subs);
    r.vec(p.idx);
    r.vec(p.vals);
    r.vec(p.stages);
    r.pod(p.n_work_stages);
    r.pod(p.scr_rows);
    r.pod(p.in_rows);
    r.pod(p.out_rows);
    r.pod(p.max_n_out);
    r.pod(p.max_n_in);
    r.vec(p.fgroups);
    r.vec(p.flevels);
    r.vec(p.fops);
    r.vec(p.fsubs);
    r.pod(p.f_max_lds_rows);
    r.pod(p.fused_ok);
    r.pod(p.f_extra_rows);
}

std::vector<unsigned char> payload_of(const PackedPlan &pk, const BuildStats &st) {
    Writer w;
    put_program(w, pk.fwd);
    put_program(w, pk.adj);
    w.vec(pk.x_off);
    w.vec(pk.y_off);
    w.vec(pk.gen_fwd.items);
    w.vec(pk.gen_fwd.task_first);
    w.vec(pk.gen_fwd.segs);
    w.vec(pk.gen_fwd.ck);
    w.vec(pk.gen_fwd.ckexp);
    w.pod(pk.gen_fwd.entries);
    w.vec(pk.gen_adj.items);
    w.vec(pk.gen_adj.task_first);
    w.vec(pk.gen_adj.segs);
    w.vec(pk.gen_adj.ck);
    w.vec(pk.gen_adj.ckexp);
    w.pod(st);
    return std::move(w.b);
}

bool read_file(const std::string &path, std::vector<unsigned char> &buf) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    f.seekg(0, std::ios::end);
    const std::streamoff n = f.tellg();
    if (n < 0) return false;
    f.seekg(0, std::ios::beg);
    buf.resize((size_t)n);
    if (n > 0) f.read(reinterpret_cast<char *>(buf.data()), n);
    return (bool)f;
}

// header check; on success `key` and the payload span are returned
int parse(const std::vector<unsigned char> &buf, std::string &key, size_t &pay_at, uint64_t &pay_len) {
    Reader r{buf.data(), buf.size()};
    char magic[8];
    for (char &c : magic) r.pod(c);
    uint32_t fmt = 0, klen = 0;
    r.pod(fmt);
    r.pod(klen);
    if (!r.ok || std::memcmp(magic, kMagic, 8) != 0 || fmt != kFormat || klen > buf.size() - r.at)
        return SHT_ERR_PLAN_CORRUPT;
    key.assign(reinterpret_cast<const char *>(buf.data() + r.at), klen);
    r.at += klen;
    uint64_t sum = 0;
    r.pod(pay_len);
    r.pod(sum);
    if (!r.ok || pay_len != buf.size() - r.at) return SHT_ERR_PLAN_CORRUPT;
    pay_at = r.at;
    if (fnv1a(buf.data() + pay_at, pay_len) != sum) return SHT_ERR_PLAN_CORRUPT;
    return SHT_OK;
}

}  // namespace

const char *cache_status_name(int status) {
    switch (status) {
        case kCacheHit: return "hit";
        case kCacheMiss: return "miss";
        case kCacheRebuilt: return "corrupt_rebuilt";
        default: return "off";
    }
}

std::string cache_key(int N, const sht_plan_opts &o) {
    std::ostringstream os;
    os.precision(17);
    os << "v" << kPlanVersion << " N=" << N << " eps=" << o.eps << " n0=" << o.n0 << " leaf=" << o.leaf
       << " rk=" << o.rk << " t=" << o.oversample << " rsvd_r=" << o.rsvd_r << " rsvd_q=" << o.rsvd_q
       << " sampling=" << o.sampling << " seed=" << o.seed << " f32_mode=" << o.f32_mode
       << " min_idbf=" << o.min_idbf << " dense_gen=" << o.dense_gen << " m=" << o.m_lo << ":" << o.m_hi
       << " id_check=" << o.id_check;
    return os.str();
}

std::string cache_path(const std::string &dir, const std::string &key) {
    const uint64_t h = fnv1a(reinterpret_cast<const unsigned char *>(key.data()), key.size());
    char name[64];
    std::snprintf(name, sizeof name, "sht_plan_%016llx.bin", (unsigned long long)h);
    std::string d = dir;
    if (!d.empty() && d.back() != '/') d += '/';
    return d + name;
}

int cache_verify(const std::string &path) {
    std::vector<unsigned char> buf;
    if (!read_file(path, buf)) return SHT_ERR_INVALID_ARG;
    std::string key;
    size_t at = 0;
    uint64_t len = 0;
    return parse(buf, key, at, len);
}

int cache_load(const std::string &path, const std::string &key, PackedPlan &pk, BuildStats &st) {
    std::vector<unsigned char> buf;
    if (!read_file(path, buf)) return SHT_ERR_INVALID_ARG;
    std::string fkey;
    size_t at = 0;
    uint64_t len = 0;
    const int rc = parse(buf, fkey, at, len);
    if (rc) return rc;
    if (fkey != key) return SHT_ERR_INVALID_ARG;
    Reader r{buf.data() + at, (size_t)len};
    PackedPlan p;
    get_program(r, p.fwd);
    get_program(r, p.adj);
    r.vec(p.x_off);
    r.vec(p.y_off);
    r.vec(p.gen_fwd.items);
    r.vec(p.gen_fwd.task_first);
    r.vec(p.gen_fwd.segs);
    r.vec(p.gen_fwd.ck);
    r.vec(p.gen_fwd.ckexp);
    r.pod(p.gen_fwd.entries);
    r.vec(p.gen_adj.items);
    r.vec(p.gen_adj.task_first);
    r.vec(p.gen_adj.segs);
    r.vec(p.gen_adj.ck);
    r.vec(p.gen_adj.ckexp);
    BuildStats s;
    r.pod(s);
    if (!r.ok || r.at != r.n) return SHT_ERR_PLAN_CORRUPT;
    pk = std::move(p);
    st = s;
    return SHT_OK;
}

int cache_store(const std::string &path, const std::string &key, const PackedPlan &pk, const BuildStats &st) {
    const std::vector<unsigned char> pay = payload_of(pk, st);
    Writer h;
    for (char c : kMagic) h.pod(c);
    h.pod(kFormat);
    h.pod((uint32_t)key.size());
    h.b.insert(h.b.end(), key.begin(), key.end());
    h.pod((uint64_t)pay.size());
    h.pod(fnv1a(pay.data(), pay.size()));
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        if (!f) return SHT_ERR_INVALID_ARG;
        f.write(reinterpret_cast<const char *>(h.b.data()), (std::streamsize)h.b.size());
        f.write(reinterpret_cast<const char *>(pay.data()), (std::streamsize)pay.size());
        if (!f) {
            std::remove(tmp.c_str());
            return SHT_ERR_INVALID_ARG;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return SHT_ERR_INVALID_ARG;
    }
    return SHT_OK;
}

}  // namespace idbf
}  // namespace sht
