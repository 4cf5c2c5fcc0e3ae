#include "costmodel.hpp"

#include <cmath>
#include <fstream>
#include <sstream>

namespace ustat {

namespace {
bool read_vec(std::istream &in, std::vector<float> &v, size_t n) {
    v.resize(n);
    for (size_t i = 0; i < n; ++i)
        if (!(in >> v[i])) return false;
    return true;
}
}  // namespace

std::string load_mlp(const std::string &path, MLPWeights &w) {
    std::ifstream in(path);
    if (!in) return "cannot open " + path;
    std::string magic;
    int ver = 0;
    if (!(in >> magic >> ver) || magic != "ustat-mlp" || ver != 1) return "not a ustat-mlp v1 file";
    if (!(in >> w.F >> w.H1 >> w.H2) || w.F < 1 || w.H1 < 1 || w.H2 < 1 || w.F > 256 ||
        w.H1 > 1024 || w.H2 > 1024)
        return "bad layer sizes";
    if (!read_vec(in, w.mean, w.F) || !read_vec(in, w.inv_std, w.F) ||
        !read_vec(in, w.W1, (size_t)w.H1 * w.F) || !read_vec(in, w.b1, w.H1) ||
        !read_vec(in, w.W2, (size_t)w.H2 * w.H1) || !read_vec(in, w.b2, w.H2) ||
        !read_vec(in, w.W3, w.H2) || !read_vec(in, w.b3, 1))
        return "truncated weights";
    for (float f : w.W1)
        if (!std::isfinite(f)) return "non-finite weight";
    return "";
}

std::string save_mlp(const std::string &path, const MLPWeights &w) {
    std::ofstream out(path);
    if (!out) return "cannot write " + path;
    out.precision(9);
    out << "ustat-mlp 1\n" << w.F << " " << w.H1 << " " << w.H2 << "\n";
    auto put = [&](const std::vector<float> &v) {
        for (float f : v) out << f << " ";
        out << "\n";
    };
    put(w.mean);
    put(w.inv_std);
    put(w.W1);
    put(w.b1);
    put(w.W2);
    put(w.b2);
    put(w.W3);
    put(w.b3);
    return out ? "" : "write failed";
}

float mlp_forward(const MLPWeights &w, const float *x) {
    std::vector<float> z(w.F), h1(w.H1), h2(w.H2);
    for (int i = 0; i < w.F; ++i) z[i] = (x[i] - w.mean[i]) * w.inv_std[i];
    for (int j = 0; j < w.H1; ++j) {
        float s = w.b1[j];
        for (int i = 0; i < w.F; ++i) s += w.W1[(size_t)j * w.F + i] * z[i];
        h1[j] = s > 0 ? s : 0;
    }
    for (int j = 0; j < w.H2; ++j) {
        float s = w.b2[j];
        for (int i = 0; i < w.H1; ++i) s += w.W2[(size_t)j * w.H1 + i] * h1[i];
        h2[j] = s > 0 ? s : 0;
    }
    float s = w.b3[0];
    for (int i = 0; i < w.H2; ++i) s += w.W3[i] * h2[i];
    return s;
}

double CostModel::score(const std::vector<float> &feat) const {
    if ((int)feat.size() != w_.F) return 0.0;
    return mlp_forward(w_, feat.data());
}

}  // namespace ustat
