// Runs every oracle entry point on small and edge-case inputs; built by
// tests/test_oracle_sanitize.py with AddressSanitizer and UBSan (host code).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int orc_total_weight(const float* w, int64_t n, double* hi, double* lo);
int orc_vose_build(const float* w, int64_t n, float* t, int32_t* alias);
int orc_sweep_build(const float* w, int64_t n, float* t, int32_t* alias);
int orc_psaplus_build(const float* w, int64_t n, int64_t block, float* t, int32_t* alias);
int64_t orc_psaplus_leftovers(const float* w, int64_t n, int64_t block);
int orc_twolevel_build(const float* w, int64_t n, int64_t block, float* tt, int32_t* at, float* t, int32_t* a);
int orc_twolevel_sample(const float* tt, const int32_t* at, const float* t, const int32_t* a, int64_t n,
                        int64_t block, uint64_t seed, uint32_t sid, uint64_t first, int64_t k, int32_t* out);
int orc_alias_sample(const float* t, const int32_t* a, int64_t n, uint64_t seed, uint32_t sid, uint64_t first,
                     int64_t k, int32_t* out);
int orc_reconstruct(const float* w, const float* t, const int32_t* a, int64_t n, double* mass, double* err);
int orc_light_t_at(const float* w, int64_t n, const int64_t* idx, int64_t m, float* t, int32_t* light);
int orc_wor_keys(const float* w, int64_t n, uint64_t seed, uint32_t sid, double* keys);
int orc_sample_wor(const float* w, int64_t n, int64_t k, uint64_t seed, uint32_t sid, int32_t* out, double* kth);
int orc_permutation(const float* w, int64_t n, uint64_t seed, uint32_t sid, int32_t* out);
int orc_os_binomial(int64_t m, double rho, uint64_t seed, uint64_t heap, uint32_t tag, int64_t* out);
int orc_os_groups(const float* w, int64_t n, int32_t* order, int32_t* gexp, int64_t* gstart, int64_t* gcount,
                  int64_t* u, int64_t* np);
int orc_os_sample(const float* w, int64_t n, int64_t k, uint64_t seed, int32_t* items, int64_t* counts,
                  int64_t* s);
}

static int run(const std::vector<float>& w) {
    const int64_t n = (int64_t)w.size();
    std::vector<float> t(n), tt(n);
    std::vector<int32_t> a(n), at(n), out(4 * n + 8);
    std::vector<double> mass(n), err(n), keys(n);
    double hi, lo, kth;
    int bad = 0;
    orc_total_weight(w.data(), n, &hi, &lo);
    if (orc_sweep_build(w.data(), n, t.data(), a.data()) == 0) {
        orc_reconstruct(w.data(), t.data(), a.data(), n, mass.data(), err.data());
        orc_alias_sample(t.data(), a.data(), n, 7, 1, 5, 4 * n, out.data());
        std::vector<int64_t> idx(n);
        std::vector<int32_t> light(n);
        for (int64_t i = 0; i < n; ++i) idx[i] = i;
        orc_light_t_at(w.data(), n, idx.data(), n, t.data(), light.data());
    }
    orc_vose_build(w.data(), n, t.data(), a.data());
    for (int64_t block : {1, 3, 64, 2048}) {
        orc_psaplus_build(w.data(), n, block, t.data(), a.data());
        orc_psaplus_leftovers(w.data(), n, block);
        const int64_t G = (n + block - 1) / block;
        std::vector<float> tg(G);
        std::vector<int32_t> ag(G);
        if (orc_twolevel_build(w.data(), n, block, tg.data(), ag.data(), t.data(), a.data()) == 0)
            orc_twolevel_sample(tg.data(), ag.data(), t.data(), a.data(), n, block, 3, 2, 0, 4 * n, out.data());
    }
    orc_wor_keys(w.data(), n, 9, 0, keys.data());
    orc_sample_wor(w.data(), n, (n + 1) / 2, 9, 0, out.data(), &kth);
    orc_permutation(w.data(), n, 9, 0, out.data());
    {  // output-sensitive sampling: groups, then samples of several sizes
        std::vector<int32_t> order(n), gexp(300), items(n);
        std::vector<int64_t> gstart(300), gcount(300), counts(n);
        int64_t u = 0, np = 0, s = 0;
        orc_os_groups(w.data(), n, order.data(), gexp.data(), gstart.data(), gcount.data(), &u, &np);
        // items and counts hold n entries, enough for min(k, n) pairs
        for (int64_t kk : {(int64_t)0, (int64_t)1, (int64_t)7, n, 4 * n, (int64_t)1 << 30})
            orc_os_sample(w.data(), n, kk, 5, items.data(), counts.data(), &s);
    }
    return bad;
}

int main() {
    uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, o[4];
    orc_philox4x32_10(c, k, o);
    int64_t x = 0;  // both binomial regimes, reflection, the degenerate cases, a bad probability
    for (int64_t m : {(int64_t)0, (int64_t)1, (int64_t)30, (int64_t)1000, (int64_t)1 << 30})
        for (double rho : {0.0, 1e-9, 0.1, 0.5, 0.97, 1.0}) orc_os_binomial(m, rho, 3, 7, 2, &x);
    orc_os_binomial(10, 1.5, 3, 7, 2, &x);
    std::vector<std::vector<float>> cases = {
        {1.0f}, {0.0f, 3.0f}, {1, 2, 3, 6}, {4, 4, 4, 4}, {0, 0, 7}, {1e-40f, 0.95f}, {1e30f, 1e-30f, 1.0f},
        {-0.0f, 1.0f, 2.0f}, {1.0f, -1.0f}, {NAN, 1.0f}, {INFINITY}, {0.0f, 0.0f}};
    std::vector<float> big(5000);
    for (int i = 0; i < 5000; ++i) big[i] = (float)((i * 2654435761u) % 1000) / 7.0f;
    cases.push_back(big);
    int bad = 0;
    for (auto& w : cases) bad += run(w);
    std::printf("oracle sanitize: %zu cases\n", cases.size());
    return bad;
}
