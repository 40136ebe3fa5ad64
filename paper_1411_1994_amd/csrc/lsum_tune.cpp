// The autotuner's decision table: per shape bucket the launch variant that ran fastest when the
// bucket was first met (every variant adds the same terms in the same order, so the choice never
// changes a result).  Decisions are kept per context and, with a tuning file, appended to it as
// "tag key choice ms0 ms1 ..." lines and read back by later contexts on a device with the same tag.
#include <cstdio>
#include <fstream>
#include <sstream>

#include "lsum_internal.h"

namespace lsum {

int Tuner::get(const std::string& key) {
    if (!enabled()) return -2;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = dec_.find(key);
    return it == dec_.end() ? -1 : it->second.choice;
}

int Tuner::put(const std::string& key, const std::vector<double>& ms) {
    int best = -1;
    for (size_t v = 0; v < ms.size(); ++v)
        if (ms[v] >= 0.0 && (best < 0 || ms[v] < ms[best])) best = (int)v;
    if (best < 0) return -1;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = dec_.find(key);
    if (it != dec_.end()) return it->second.choice;   // another thread decided first
    dec_[key] = Entry{best, ms};
    if (!path_.empty()) {
        std::ofstream f(path_, std::ios::app);
        if (f) {
            f << tag_ << ' ' << key << ' ' << best;
            for (double t : ms) f << ' ' << t;
            f << '\n';
        }
    }
    return best;
}

int Tuner::use_file(const std::string& path) {
    std::lock_guard<std::mutex> lk(mu_);
    path_ = path;
    std::ifstream f(path);
    if (!f) return LSUM_OK;   // created on the first decision
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string tag, key;
        int choice = -1;
        if (!(in >> tag >> key >> choice) || tag != tag_ || choice < 0) continue;
        std::vector<double> ms;
        double t;
        while (in >> t) ms.push_back(t);
        if (choice >= (int)ms.size()) continue;
        dec_[key] = Entry{choice, ms};
    }
    return LSUM_OK;
}

std::string Tuner::json() {
    std::lock_guard<std::mutex> lk(mu_);
    std::ostringstream o;
    o.precision(6);
    o << "{\"device\":\"" << tag_ << "\",\"file\":\"" << path_ << "\",\"enabled\":" << on_.load() << ",\"decisions\":{";
    bool first = true;
    for (auto& kv : dec_) {
        o << (first ? "" : ",") << "\"" << kv.first << "\":{\"choice\":" << kv.second.choice << ",\"ms\":[";
        for (size_t k = 0; k < kv.second.ms.size(); ++k) o << (k ? "," : "") << kv.second.ms[k];
        o << "]}";
        first = false;
    }
    o << "}}";
    return o.str();
}

}  // namespace lsum
