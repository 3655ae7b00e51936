// LDS capacity of the segment-test tile for every launch shape the library accepts:
// each wave's pre-test queue segment must hold every pixel the wave can append.
// Host build of the library's own layout code (of_plan.h); prints one line per failure
// and "ok <shapes>" at the end.
#include <cstdio>

#include "../../paper_2506_07164_amd/csrc/of_plan.h"

int main() {
  using namespace ofk;
  int shapes = 0, bad = 0;
  for (int words = 1; words <= 4; ++words)
    for (int rows = 4; rows <= 64; ++rows) {
      Tune t{};
      t.mark_words = words;
      t.mark_rows = rows;
      const MarkLds m = mark_lds(t);
      ++shapes;
      // Wave w of the 4 takes tile rows w, w + 4, ...; a row holds 64 * words pixels.
      int worst = 0;
      for (int w = 0; w < 4; ++w) {
        int n = 0;
        for (int r = w; r < rows; r += 4) n += 64 * words;
        if (n > worst) worst = n;
      }
      const bool fits = m.qseg >= worst && m.off_queue + 2 * 4 * m.qseg <= m.off_bml &&
                        m.off_queue >= m.pitch * m.rows && m.pitch >= 64 * words + 7 &&
                        m.rows >= rows + 6;
      if (!fits) {
        ++bad;
        std::printf("mark_words %d mark_rows %d: queue segment %d < %d appends\n", words, rows,
                    m.qseg, worst);
      }
    }
  std::printf("%s %d\n", bad ? "fail" : "ok", shapes);
  return bad ? 1 : 0;
}
