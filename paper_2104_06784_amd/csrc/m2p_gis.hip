// m2p_gis.hip -- ESRI ASCII grid input and output (host only).
//
// The paper's tool takes its DEM from GIS systems as ASCII grids and converts
// the computed thickness, solid fraction and velocities back to that form
// (Sect. 1; Sect. 3.1.2, Stages 1 and 3).  The ESRI ASCII grid is
// the common text form: a header of keyword/value lines (ncols, nrows,
// xllcorner or xllcenter, yllcorner or yllcenter, cellsize, optional
// NODATA_value), then nrows lines of ncols values, northernmost row first.
// Arrays at the C ABI are row-major with row 0 at the southern edge (y
// increasing with the row index), so rows are flipped on read and write.
#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "m2p.h"
#include "m2p_host.h"

namespace {

struct Header {
    long ncols = -1, nrows = -1;
    double x = NAN, y = NAN, cell = NAN, nodata = -9999.0;
    bool xcenter = false, ycenter = false, has_nodata = false;
};

bool iequal(const char* a, const char* b)
{
    for (; *a && *b; a++, b++)
        if (std::tolower((unsigned char)*a) != std::tolower((unsigned char)*b)) return false;
    return *a == *b;
}

// Reads the header; leaves f at the first data value.
int read_header(FILE* f, Header& h)
{
    char key[64];
    for (;;) {
        const long pos = std::ftell(f);
        if (std::fscanf(f, " %63s", key) != 1) return m2p::fail(M2P_EINVAL, "ESRI grid: truncated header");
        if (!std::isalpha((unsigned char)key[0])) {
            std::fseek(f, pos, SEEK_SET);
            break;
        }
        double v;
        if (std::fscanf(f, " %lf", &v) != 1) return m2p::fail(M2P_EINVAL, std::string("ESRI grid: no value for ") + key);
        if (iequal(key, "ncols"))
            h.ncols = (long)v;
        else if (iequal(key, "nrows"))
            h.nrows = (long)v;
        else if (iequal(key, "xllcorner"))
            h.x = v;
        else if (iequal(key, "xllcenter")) {
            h.x = v;
            h.xcenter = true;
        } else if (iequal(key, "yllcorner"))
            h.y = v;
        else if (iequal(key, "yllcenter")) {
            h.y = v;
            h.ycenter = true;
        } else if (iequal(key, "cellsize"))
            h.cell = v;
        else if (iequal(key, "nodata_value")) {
            h.nodata = v;
            h.has_nodata = true;
        } else
            return m2p::fail(M2P_EINVAL, std::string("ESRI grid: unknown header key ") + key);
    }
    if (h.ncols < 1 || h.nrows < 1 || h.ncols > (1L << 20) || h.nrows > (1L << 20))
        return m2p::fail(M2P_EINVAL, "ESRI grid: bad ncols / nrows");
    if (!(h.cell > 0.0) || !std::isfinite(h.x) || !std::isfinite(h.y))
        return m2p::fail(M2P_EINVAL, "ESRI grid: bad cellsize or lower-left corner");
    return M2P_OK;
}

}  // namespace

extern "C" int m2p_esri_read(const char* path, m2p_grid* g, double* x0, double* y0, double* nodata, double* values,
                             size_t capacity)
{
    if (!path || !g) return m2p::fail(M2P_EINVAL, "NULL argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return m2p::fail(M2P_EIO, std::string("cannot open ") + path + ": " + std::strerror(errno));
    Header h;
    int rc = read_header(f, h);
    if (rc == M2P_OK) {
        g->nx = (int32_t)h.ncols;
        g->ny = (int32_t)h.nrows;
        g->dx = g->dy = h.cell;
        // lower-left cell corner
        if (x0) *x0 = h.xcenter ? h.x - 0.5 * h.cell : h.x;
        if (y0) *y0 = h.ycenter ? h.y - 0.5 * h.cell : h.y;
        if (nodata) *nodata = h.has_nodata ? h.nodata : NAN;
        const size_t n = (size_t)h.ncols * (size_t)h.nrows;
        if (values) {
            if (capacity < n) {
                rc = m2p::fail(M2P_EINVAL, "ESRI grid: values array smaller than ncols * nrows");
            } else {
                for (long r = 0; r < h.nrows && rc == M2P_OK; r++) {
                    double* row = values + (size_t)(h.nrows - 1 - r) * h.ncols;  // file row 0 is the north edge
                    for (long c = 0; c < h.ncols; c++) {
                        if (std::fscanf(f, " %lf", &row[c]) != 1) {
                            rc = m2p::fail(M2P_EINVAL, "ESRI grid: fewer values than ncols * nrows");
                            break;
                        }
                        // a cell without data is NaN, never a number: a DEM or
                        // a thickness holding one is rejected by m2p_create /
                        // m2p_set_state instead of becoming a pit of -9999 m
                        if (h.has_nodata && row[c] == h.nodata) row[c] = NAN;
                    }
                }
                double extra;
                if (rc == M2P_OK && std::fscanf(f, " %lf", &extra) == 1)
                    rc = m2p::fail(M2P_EINVAL, "ESRI grid: more values than ncols * nrows");
            }
        }
    }
    std::fclose(f);
    return rc;
}

extern "C" int m2p_esri_write(const char* path, const m2p_grid* g, double x0, double y0, double nodata,
                              const double* values)
{
    if (!path || !g || !values) return m2p::fail(M2P_EINVAL, "NULL argument");
    if (g->nx < 1 || g->ny < 1 || !(g->dx > 0.0) || g->dx != g->dy || !std::isfinite(x0) || !std::isfinite(y0))
        return m2p::fail(M2P_EINVAL, "ESRI grid needs nx, ny >= 1 and square cells dx = dy > 0");
    FILE* f = std::fopen(path, "w");
    if (!f) return m2p::fail(M2P_EIO, std::string("cannot create ") + path + ": " + std::strerror(errno));
    std::fprintf(f, "ncols %d\nnrows %d\nxllcorner %.17g\nyllcorner %.17g\ncellsize %.17g\nNODATA_value %.17g\n",
                 g->nx, g->ny, x0, y0, g->dx, nodata);
    for (int r = 0; r < g->ny; r++) {
        const double* row = values + (size_t)(g->ny - 1 - r) * g->nx;
        for (int c = 0; c < g->nx; c++) {
            const double v = std::isfinite(row[c]) ? row[c] : nodata;
            std::fprintf(f, c ? " %.17g" : "%.17g", v);
        }
        std::fputc('\n', f);
    }
    const bool bad = std::ferror(f) != 0;
    if (std::fclose(f) != 0 || bad) return m2p::fail(M2P_EIO, std::string("write failed: ") + path);
    return M2P_OK;
}
