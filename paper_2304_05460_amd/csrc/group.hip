// Recorder of deferred launches and the grouped replay (declarations and the
// scheme in group.h).
#include "group.h"

namespace afn {

Recorder *&recorder()
{
    static thread_local Recorder *r = nullptr;
    return r;
}

afn_status defer(hipStream_t s, std::function<hipError_t(hipStream_t)> f)
{
    if (Recorder *r = recorder()) {
        DeferredOp op;
        op.run = std::move(f);
        r->ops.push_back(std::move(op));
        return AFN_OK;
    }
    AFN_HIP(f(s));
    return AFN_OK;
}

afn_status replay_grouped(Recorder *const *recs, int G, hipStream_t s, char *merged)
{
    for (int g = 0; g < G; ++g) merged[g] = 0;
    std::vector<char> seen(G, 0);
    std::vector<int> part, cls;
    std::vector<char> used;
    std::vector<const DeferredOp *> slice;
    slice.reserve(kGroupMax);
    for (int g0 = 0; g0 < G; ++g0) {
        if (seen[g0]) continue;
        // the recordings as long as g0's
        const size_t nops = recs[g0]->ops.size();
        part.clear();
        for (int g = g0; g < G; ++g)
            if (!seen[g] && recs[g]->ops.size() == nops) {
                part.push_back(g);
                seen[g] = 1;
            }
        const int P = (int)part.size();
        for (size_t j = 0; j < nops; ++j) {
            used.assign(P, 0);
            for (int a = 0; a < P; ++a) {
                if (used[a]) continue;
                const DeferredOp &op = recs[part[a]]->ops[j];
                used[a] = 1;
                cls.assign(1, part[a]);
                if (op.group)
                    for (int b = a + 1; b < P; ++b)
                        if (!used[b] && recs[part[b]]->ops[j].group == op.group) {
                            cls.push_back(part[b]);
                            used[b] = 1;
                        }
                if (cls.size() == 1) {
                    AFN_HIP(op.run(s));
                    continue;
                }
                for (size_t c0 = 0; c0 < cls.size(); c0 += kGroupMax) {
                    slice.clear();
                    for (size_t c = c0; c < cls.size() && c < c0 + kGroupMax; ++c) {
                        slice.push_back(&recs[cls[c]]->ops[j]);
                        merged[cls[c]] = 1;
                    }
                    AFN_HIP(op.group(slice.data(), (int)slice.size(), s));
                }
            }
        }
    }
    return AFN_OK;
}

}  // namespace afn
