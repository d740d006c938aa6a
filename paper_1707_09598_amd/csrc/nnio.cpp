// nnio.cpp -- host side of the learned preconditioner's network: seeded
// initialisation of the parameters and a checked file format for them.
//
// File layout (little endian): the 8 bytes "IGANNv01", int32 nlayers, int32
// head, int32 channels[nlayers + 1], int64 count, float params[count], then
// the CRC-32 (IEEE 802.3 polynomial, reflected, initial and final value
// 0xffffffff) of every preceding byte.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "iga_nn.h"
#include "plan.hpp"

using igasg::set_error;

namespace {

constexpr char kMagic[8] = {'I', 'G', 'A', 'N', 'N', 'v', '0', '1'};
constexpr int kMaxLayers = 8;

bool net_ok(const int* channels, int nlayers) {
    if (!channels || nlayers < 1 || nlayers > kMaxLayers) return false;
    for (int l = 0; l <= nlayers; ++l)
        if (channels[l] < 1 || channels[l] > 1024) return false;
    return true;
}

int64_t count_of(const int* channels, int nlayers) {
    int64_t c = 0;
    for (int l = 0; l < nlayers; ++l) c += static_cast<int64_t>(channels[l + 1]) * (channels[l] * 27 + 1);
    return c;
}

uint32_t crc32(const unsigned char* p, size_t n, uint32_t crc = 0xffffffffu) {
    for (size_t i = 0; i < n; ++i) {
        crc ^= p[i];
        for (int b = 0; b < 8; ++b) crc = (crc >> 1) ^ (0xedb88320u & (0u - (crc & 1u)));
    }
    return crc;
}

// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", 2014): the state advances by the golden-ratio increment and
// the output is a 64-bit finaliser of the state.
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    // uniform in (0, 1): the top 53 bits, shifted by half an ulp
    double uniform() { return (static_cast<double>(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    // standard normal by the Box-Muller transform
    double normal() {
        const double u = uniform(), v = uniform();
        return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
    }
};

}  // namespace

extern "C" {

iga_status iga_nn_init(const int* channels, int nlayers, uint64_t seed, float* params_host) {
    if (!net_ok(channels, nlayers) || !params_host) {
        set_error("iga_nn_init: invalid network description");
        return IGA_ERR_INVALID_ARG;
    }
    SplitMix64 rng{seed};
    float* p = params_host;
    for (int l = 0; l < nlayers; ++l) {
        const int cin = channels[l], cout = channels[l + 1];
        const double sd = std::sqrt(2.0 / (27.0 * cin));  // He initialisation for ReLU layers
        const int64_t nw = static_cast<int64_t>(cout) * cin * 27;
        for (int64_t i = 0; i < nw; ++i) {
            const double v = rng.normal() * sd;
            p[i] = l == nlayers - 1 ? 0.0f : static_cast<float>(v);  // last layer 0: the plain preconditioner
        }
        p += nw;
        for (int c = 0; c < cout; ++c) *p++ = 0.0f;
    }
    return IGA_OK;
}

iga_status iga_nn_save(const char* path, const int* channels, int nlayers, int head, const float* params_host) {
    if (!path || !net_ok(channels, nlayers) || !params_host || head < 0 || head > 1) {
        set_error("iga_nn_save: invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    std::vector<unsigned char> buf(kMagic, kMagic + 8);
    auto put = [&](const void* v, size_t n) {
        const unsigned char* c = static_cast<const unsigned char*>(v);
        buf.insert(buf.end(), c, c + n);
    };
    const int32_t nl = nlayers, hd = head;
    put(&nl, 4);
    put(&hd, 4);
    for (int l = 0; l <= nlayers; ++l) {
        const int32_t c = channels[l];
        put(&c, 4);
    }
    const int64_t count = count_of(channels, nlayers);
    put(&count, 8);
    put(params_host, sizeof(float) * static_cast<size_t>(count));
    const uint32_t crc = crc32(buf.data(), buf.size()) ^ 0xffffffffu;
    put(&crc, 4);
    FILE* f = std::fopen(path, "wb");
    if (!f) {
        set_error("iga_nn_save: cannot open %s", path);
        return IGA_ERR_INVALID_ARG;
    }
    const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
    const int rc = std::fclose(f);
    if (w != buf.size() || rc != 0) {
        set_error("iga_nn_save: write to %s failed", path);
        return IGA_ERR_INVALID_ARG;
    }
    return IGA_OK;
}

iga_status iga_nn_load(const char* path, int* channels, int* nlayers, int* head, float* params_host,
                       int64_t capacity) {
    if (!path || !nlayers) {
        set_error("iga_nn_load: invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        set_error("iga_nn_load: cannot open %s", path);
        return IGA_ERR_INVALID_ARG;
    }
    std::vector<unsigned char> buf;
    unsigned char tmp[4096];
    size_t r;
    while ((r = std::fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + r);
    std::fclose(f);
    auto bad = [&](const char* what) {
        set_error("iga_nn_load: %s: %s", path, what);
        return IGA_ERR_INVALID_ARG;
    };
    if (buf.size() < 8 + 8 + 8 + 4 || std::memcmp(buf.data(), kMagic, 8) != 0) return bad("not a network file");
    uint32_t crc;
    std::memcpy(&crc, buf.data() + buf.size() - 4, 4);
    if ((crc32(buf.data(), buf.size() - 4) ^ 0xffffffffu) != crc) return bad("checksum mismatch");
    size_t o = 8;
    int32_t nl, hd;
    std::memcpy(&nl, buf.data() + o, 4);
    std::memcpy(&hd, buf.data() + o + 4, 4);
    o += 8;
    if (nl < 1 || nl > kMaxLayers || buf.size() < o + 4 * (nl + 1) + 8 + 4) return bad("bad header");
    int ch[kMaxLayers + 1];
    for (int l = 0; l <= nl; ++l) std::memcpy(&ch[l], buf.data() + o + 4 * l, 4);
    o += 4 * (nl + 1);
    int64_t count;
    std::memcpy(&count, buf.data() + o, 8);
    o += 8;
    if (!net_ok(ch, nl) || count != count_of(ch, nl) || buf.size() != o + 4 * static_cast<size_t>(count) + 4)
        return bad("inconsistent sizes");
    *nlayers = nl;
    if (head) *head = hd;
    if (channels)
        for (int l = 0; l <= nl; ++l) channels[l] = ch[l];
    if (params_host) {
        if (capacity < count) return bad("parameter buffer too small");
        std::memcpy(params_host, buf.data() + o, 4 * static_cast<size_t>(count));
    }
    return IGA_OK;
}

}  // extern "C"
