// Training the learned cost model from a measurement database: the JSON-lines
// file the autotuner and the group-measurement entry point append to (one
// line per timed configuration: its measured time and its 40 model
// features).  The network predicts log(measured microseconds); features and
// target are standardised on the training rows (stored in the model).
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "wt_cost.h"
#include "wt_mlp.h"

namespace wt {

namespace {

// Value after `"key":` on a JSON line; npos when the key is absent.
size_t value_pos(const std::string& line, const char* key) {
    std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return p;
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return p;
    ++p;
    while (p < line.size() && line[p] == ' ') ++p;
    return p;
}

// A JSON number at `p` (null, inf and nan read as non-finite); advances p.
double number_at(const std::string& line, size_t& p) {
    while (p < line.size() && line[p] == ' ') ++p;
    if (line.compare(p, 4, "null") == 0) {
        p += 4;
        return NAN;
    }
    const char* s = line.c_str() + p;
    char* end = nullptr;
    double v = std::strtod(s, &end);  // also reads inf / -inf / nan
    if (end == s) return NAN;
    p += (size_t)(end - s);
    return v;
}

// Numbers of the array value of `key` (empty when absent or malformed).
std::vector<double> array_of(const std::string& line, const char* key, bool* ok) {
    std::vector<double> out;
    *ok = false;
    size_t p = value_pos(line, key);
    if (p == std::string::npos || p >= line.size() || line[p] != '[') return out;
    ++p;
    while (p < line.size()) {
        while (p < line.size() && line[p] == ' ') ++p;
        if (p < line.size() && line[p] == ']') {
            *ok = true;
            return out;
        }
        size_t before = p;
        out.push_back(number_at(line, p));
        if (p == before) return out;
        while (p < line.size() && line[p] == ' ') ++p;
        if (p < line.size() && line[p] == ',') ++p;
    }
    return out;
}

}  // namespace

int read_measure_db(const std::string& path, std::vector<float>& x, std::vector<float>& t) {
    std::ifstream f(path);
    if (!f) fail(WT_E_INVALID, "cannot open measurement database " + path);
    std::string line;
    int rows = 0;
    while (std::getline(f, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        size_t p = value_pos(line, "measured_us");
        if (p == std::string::npos) fail(WT_E_INVALID, "measurement line without measured_us: " + line.substr(0, 80));
        double us = number_at(line, p);
        size_t q = value_pos(line, "pred_us");
        double pred = q == std::string::npos ? NAN : number_at(line, q);
        bool fok = false, tok = false;
        std::vector<double> feats = array_of(line, "features", &fok);
        std::vector<double> terms = array_of(line, "terms", &tok);
        // usable rows: a positive finite time, all 40 features finite, and
        // the analytical model's quantities defined (a configuration the
        // model deems infeasible has them null)
        bool ok = std::isfinite(us) && us > 0 && fok && (int)feats.size() == kNumFeatures && std::isfinite(pred) &&
                  tok;
        for (double v : feats) ok = ok && std::isfinite(v);
        for (double v : terms) ok = ok && std::isfinite(v);
        if (!ok) continue;
        for (double v : feats) x.push_back((float)v);
        t.push_back((float)std::log(us));
        ++rows;
    }
    return rows;
}

void train_model_from_db(const std::string& db, const std::string& out_model, hipStream_t stream) {
    std::vector<float> x, t;
    int n = read_measure_db(db, x, t);
    if (n < 2) fail(WT_E_INVALID, "measurement database holds fewer than two usable rows");
    Mlp m({kNumFeatures, 128, 128, 128, 1}, 1);
    if (stream) m.use_stream(stream);
    m.train(x.data(), t.data(), n, 200, 256, 1e-3f, 1);
    m.save(out_model);
}

}  // namespace wt
