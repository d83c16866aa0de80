// Concatenation of the per-kernel schedule tables into one id space.
#include "registry.h"

namespace tg {

namespace {
constexpr int kParts = 4;
struct Table {
    const SchedDesc* parts[kParts];
    int counts[kParts];
    int total;
    Table()
    {
        parts[0] = tile_schedules(&counts[0]);
        parts[1] = scaled_schedules(&counts[1]);
        parts[2] = packed_schedules(&counts[2]);
        parts[3] = inplace_schedules(&counts[3]);
        total = counts[0] + counts[1] + counts[2] + counts[3];
    }
};

const Table& table()
{
    static const Table t;
    return t;
}
}  // namespace

int num_schedules() { return table().total; }

const SchedDesc& schedule(int id)
{
    const Table& t = table();
    for (int p = 0; p < kParts; ++p) {
        if (id < t.counts[p]) return t.parts[p][id];
        id -= t.counts[p];
    }
    return t.parts[0][0];  // callers check the id range first
}

int packed_index(int id)
{
    const Table& t = table();
    const int first = t.counts[0] + t.counts[1];
    return (id >= first && id < first + t.counts[2]) ? id - first : -1;
}

}  // namespace tg
