// Learned cost model for elimination orders: a small MLP mapping the
// features of a lowered program (plan.cpp, program_features) to a predicted
// log run time.  Host inference only; training runs on the GPU with the
// engine's own MLP kernels (mlp.hip).
#pragma once

#include <string>
#include <vector>

#include "plan.hpp"

namespace ustat {

struct MLPWeights {
    int F = 0, H1 = 0, H2 = 0;
    std::vector<float> mean, inv_std;  // input standardisation, size F
    std::vector<float> W1, b1;         // H1 x F, H1
    std::vector<float> W2, b2;         // H2 x H1, H2
    std::vector<float> W3, b3;         // 1 x H2, 1
};

// Text format, whitespace separated:
//   ustat-mlp 1  F H1 H2  mean[F] inv_std[F]  W1 b1 W2 b2 W3 b3  (row-major)
std::string load_mlp(const std::string &path, MLPWeights &w);
std::string save_mlp(const std::string &path, const MLPWeights &w);
float mlp_forward(const MLPWeights &w, const float *x);

// Thread-local detail message returned by ustat_last_error().
void set_last_error(const std::string &msg);

class CostModel : public OrderScorer {
public:
    // Loads weights; a model for another feature count is rejected.
    std::string load(const std::string &path) {
        std::string e = load_mlp(path, w_);
        if (e.empty() && w_.F != kOrderFeatures)
            e = "cost model has " + std::to_string(w_.F) + " inputs; the order features number " +
                std::to_string(kOrderFeatures);
        return e;
    }
    double score(const std::vector<float> &feat) const override;
    const MLPWeights &weights() const { return w_; }

private:
    MLPWeights w_;
};

}  // namespace ustat
