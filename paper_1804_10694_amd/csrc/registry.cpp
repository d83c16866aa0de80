// Concatenation of the per-kernel schedule tables into one id space.
#include "registry.h"

namespace tg {

namespace {
struct Table {
    const SchedDesc* parts[2];
    int counts[2];
    int total;
    Table()
    {
        parts[0] = tile_schedules(&counts[0]);
        parts[1] = scaled_schedules(&counts[1]);
        total = counts[0] + counts[1];
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
    for (int p = 0; p < 2; ++p) {
        if (id < t.counts[p]) return t.parts[p][id];
        id -= t.counts[p];
    }
    return t.parts[0][0];  // callers check the id range first
}

}  // namespace tg
