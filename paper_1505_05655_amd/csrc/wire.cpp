// TCP front end of the client-server framework (§II of the paper, header
// template of Fig. 3): clients send a 260-byte header and their input data;
// the server runs the task on the GPU and returns a header of the same layout
// followed by the result.
//
// One accept thread and one thread per connection. LUT-correction jobs of all
// connections are handed to one rc_server, so requests that arrive while
// others run share its persistent launches (continuous batching); their
// buffers are pinned, so the kernel writes the result straight into the
// buffer this thread then sends. Demosaicing and fits run on a stream of the
// connection. Requests are parsed and bounded before any byte of data is
// accepted; a malformed header is answered and the connection closed (its
// data length is unknown).
#include <arpa/inet.h>
#include <hip/hip_runtime_api.h>
#include <netinet/in.h>
#include <poll.h>
#include <sys/socket.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <list>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "rc.h"
#include "runtime.h"

namespace rc {
namespace {

constexpr size_t kTaskLen = 29, kFlagOff = 29, kParamOff = 30, kParamLen = 200, kOutOff = 230,
                 kOutLen = 30;

const char* kTaskNames[] = {nullptr,     "LUT_CORRECTION", "BILINEAR_DEMOSAIC",
                            "LSQ_FIT",   "GPU_INFO",       "GRADIENT_DEMOSAIC"};

const char* status_name(rc_status s) {
    switch (s) {
        case RC_OK: return "RC_OK";
        case RC_EINVAL: return "RC_EINVAL";
        case RC_ENOMEM: return "RC_ENOMEM";
        case RC_EHIP: return "RC_EHIP";
        case RC_EBUSY: return "RC_EBUSY";
        case RC_ECLOSED: return "RC_ECLOSED";
    }
    return "RC_UNKNOWN";
}

// Copies a NUL-padded text field; false if a byte after the first NUL is not NUL.
bool text_field(const uint8_t* h, size_t off, size_t len, char* out) {
    size_t n = 0;
    while (n < len && h[off + n] != 0) ++n;
    for (size_t k = n; k < len; ++k)
        if (h[off + k] != 0) return false;
    std::memcpy(out, h + off, n);
    out[n] = 0;
    return true;
}

bool mul_u64(uint64_t a, uint64_t b, uint64_t* r) { return !__builtin_mul_overflow(a, b, r); }

// Parameter string: key=value pairs, comma separated, values decimal integers.
struct Params {
    std::vector<std::pair<std::string, int64_t>> kv;
    bool get(const char* key, int64_t* v) const {
        for (auto& p : kv)
            if (p.first == key) {
                *v = p.second;
                return true;
            }
        return false;
    }
};

bool parse_params(const char* s, Params* out) {
    const char* p = s;
    while (*p) {
        const char* eq = std::strchr(p, '=');
        const char* end = std::strchr(p, ',');
        if (!end) end = p + std::strlen(p);
        if (!eq || eq > end || eq == p) return false;
        std::string key(p, eq - p);
        const char* v = eq + 1;
        if (v == end) return false;
        int64_t x = 0;
        for (const char* c = v; c < end; ++c) {
            if (*c < '0' || *c > '9') return false;
            if (x > (INT64_MAX - 9) / 10) return false;
            x = x * 10 + (*c - '0');
        }
        for (auto& q : out->kv)
            if (q.first == key) return false;  // duplicate
        out->kv.push_back({key, x});
        p = *end ? end + 1 : end;
        if (*end && !*p) return false;  // trailing comma
    }
    return true;
}

bool only_keys(const Params& ps, std::initializer_list<const char*> keys) {
    for (auto& p : ps.kv) {
        bool ok = false;
        for (const char* k : keys) ok |= p.first == k;
        if (!ok) return false;
    }
    return true;
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_wire_parse(const uint8_t* h, rc_wire_request* r) {
    if (!h || !r) return RC_EINVAL;
    std::memset(r, 0, sizeof *r);
    if (!text_field(h, 0, kTaskLen, r->task_flag) ||
        !text_field(h, kParamOff, kParamLen, r->params) ||
        !text_field(h, kOutOff, kOutLen, r->out_name))
        return RC_EINVAL;
    for (int t = 1; t <= 5; ++t)
        if (std::strcmp(r->task_flag, kTaskNames[t]) == 0) r->task = t;
    if (!r->task) return RC_EINVAL;
    const uint8_t flag = h[kFlagOff];
    if (flag != '+' && flag != 0) return RC_EINVAL;
    r->has_data = flag == '+';
    Params ps;
    if (!parse_params(r->params, &ps)) return RC_EINVAL;
    const int64_t I32 = INT32_MAX;
    uint64_t in = 0, res = 0, a = 0, b = 0;
    switch (r->task) {
        case RC_TASK_LUT_CORRECTION: {
            int64_t lut = 0;
            if (!only_keys(ps, {"bands", "lines", "detectors", "levels", "lut"}) ||
                !ps.get("bands", &r->bands) || !ps.get("lines", &r->lines) ||
                !ps.get("detectors", &r->detectors) || !ps.get("levels", &r->levels))
                return RC_EINVAL;
            ps.get("lut", &lut);
            if (r->bands < 1 || r->bands > I32 || r->detectors < 1 || r->detectors > I32 ||
                r->lines > I32 * (int64_t)64 || r->levels < RC_LEVELS_MIN ||
                r->levels > RC_LEVELS_MAX || lut > 1)
                return RC_EINVAL;
            r->want_lut = (int32_t)lut;
            const uint64_t rows = (uint64_t)r->bands * (uint64_t)r->detectors;
            if (!mul_u64(rows, 32, &a) || !mul_u64(rows, (uint64_t)r->lines, &b) ||
                !mul_u64(b, 2, &b) || __builtin_add_overflow(a, b, &in))
                return RC_EINVAL;
            res = b;
            if (lut) {
                uint64_t l = 0;
                if (!mul_u64(rows, (uint64_t)r->levels * 2, &l) ||
                    __builtin_add_overflow(res, l, &res))
                    return RC_EINVAL;
            }
            break;
        }
        case RC_TASK_BILINEAR_DEMOSAIC:
        case RC_TASK_GRADIENT_DEMOSAIC:
            if (!only_keys(ps, {"images", "height", "width"}) || !ps.get("images", &r->images) ||
                !ps.get("height", &r->height) || !ps.get("width", &r->width))
                return RC_EINVAL;
            if (r->images < 1 || r->images > I32 ||
                r->height < (r->task == RC_TASK_GRADIENT_DEMOSAIC ? 4 : 2) || r->height > I32 ||
                r->height % 2 || r->width < 4 || r->width > I32 || r->width % 4)
                return RC_EINVAL;
            if (!mul_u64((uint64_t)r->images, (uint64_t)r->height, &a) ||
                !mul_u64(a, (uint64_t)r->width, &a) || !mul_u64(a, 2, &in) ||
                !mul_u64(in, 3, &res))
                return RC_EINVAL;
            break;
        case RC_TASK_LSQ_FIT:
            if (!only_keys(ps, {"bands", "points", "detectors", "order"}) ||
                !ps.get("bands", &r->bands) || !ps.get("points", &r->points) ||
                !ps.get("detectors", &r->detectors) || !ps.get("order", &r->order))
                return RC_EINVAL;
            if (r->bands < 1 || r->bands > I32 || r->detectors < 1 || r->detectors > I32 ||
                r->order > 3 || r->points < r->order + 1 || r->points > I32)
                return RC_EINVAL;
            if (!mul_u64((uint64_t)r->bands, (uint64_t)r->points, &a) ||
                !mul_u64(a, (uint64_t)r->detectors, &b) || !mul_u64(b, 8, &b) ||
                !mul_u64(a, 8, &a) || __builtin_add_overflow(a, b, &in) ||
                !mul_u64((uint64_t)r->bands * (uint64_t)r->detectors, 32, &res))
                return RC_EINVAL;
            break;
        case RC_TASK_GPU_INFO:
            if (!ps.kv.empty()) return RC_EINVAL;
            in = 0;
            res = 0;  // known once the listing is written
            break;
    }
    if ((in > 0) != (r->has_data != 0)) return RC_EINVAL;
    r->data_bytes = in;
    r->result_bytes = res;
    return RC_OK;
}

// One client connection: its socket (-1 once closed), its thread, and whether
// the thread has finished (then the acceptor joins and forgets it).
struct rc_wire_conn {
    int fd = -1;
    std::atomic<bool> done{false};
    std::thread thread;
};

struct rc_wire {
    int fd = -1;
    int port = 0;
    int device = 0;
    rc_wire_opts opts{};
    rc_server* srv = nullptr;
    std::atomic<bool> stopping{false};
    std::thread acceptor;
    std::mutex mu;
    std::list<rc_wire_conn> conns;  // element addresses stay valid while listed
};

namespace rc {
namespace {

bool recv_all(int fd, void* buf, size_t n, bool* clean_eof) {
    char* p = (char*)buf;
    size_t got = 0;
    if (clean_eof) *clean_eof = false;
    while (got < n) {
        const ssize_t k = ::recv(fd, p + got, n - got, 0);
        if (k == 0) {
            if (clean_eof && got == 0) *clean_eof = true;
            return false;
        }
        if (k < 0) {
            if (errno == EINTR) continue;
            return false;
        }
        got += (size_t)k;
    }
    return true;
}

bool send_all(int fd, const void* buf, size_t n) {
    const char* p = (const char*)buf;
    while (n) {
        const ssize_t k = ::send(fd, p, n, MSG_NOSIGNAL);
        if (k < 0) {
            if (errno == EINTR) continue;
            return false;
        }
        p += k;
        n -= (size_t)k;
    }
    return true;
}

bool reply(int fd, const uint8_t* req_header, rc_status st, const void* data, uint64_t bytes) {
    uint8_t h[RC_WIRE_HEADER_BYTES];
    std::memset(h, 0, sizeof h);
    std::memcpy(h, req_header, kTaskLen);                 // task flag echoed
    std::memcpy(h + kOutOff, req_header + kOutOff, kOutLen);  // output file name echoed
    if (st != RC_OK) bytes = 0;
    h[kFlagOff] = bytes ? '+' : 0;
    std::snprintf((char*)h + kParamOff, kParamLen, "status=%s,bytes=%llu", status_name(st),
                  (unsigned long long)bytes);
    return send_all(fd, h, sizeof h) && (!bytes || send_all(fd, data, (size_t)bytes));
}

std::string xml_escape(const char* s) {
    std::string o;
    for (; *s; ++s) {
        if (*s == '&') o += "&amp;";
        else if (*s == '<') o += "&lt;";
        else if (*s == '>') o += "&gt;";
        else o += *s;
    }
    return o;
}

// §IV: the remote GPU information utility, as an XML listing.
rc_status gpu_info(std::string* xml) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return RC_EHIP;
    std::string x = "<?xml version=\"1.0\"?>\n<gpus count=\"" + std::to_string(n) + "\">\n";
    for (int d = 0; d < n; ++d) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d) != hipSuccess) return RC_EHIP;
        char buf[2048];
        std::snprintf(
            buf, sizeof buf,
            "  <gpu index=\"%d\">\n    <name>%s</name>\n    <arch>%s</arch>\n"
            "    <wavefront_size>%d</wavefront_size>\n"
            "    <total_constant_memory>%zu</total_constant_memory>\n"
            "    <total_global_memory>%zu</total_global_memory>\n"
            "    <shared_memory_per_block>%zu</shared_memory_per_block>\n"
            "    <clock_rate_khz>%d</clock_rate_khz>\n"
            "    <multiprocessor_count>%d</multiprocessor_count>\n"
            "    <registers_per_block>%d</registers_per_block>\n"
            "    <max_threads_per_block>%d</max_threads_per_block>\n"
            "    <max_grid_size>%d,%d,%d</max_grid_size>\n"
            "    <max_threads_dim>%d,%d,%d</max_threads_dim>\n  </gpu>\n",
            d, xml_escape(p.name).c_str(), xml_escape(p.gcnArchName).c_str(), p.warpSize,
            (size_t)p.totalConstMem, (size_t)p.totalGlobalMem, (size_t)p.sharedMemPerBlock,
            p.clockRate, p.multiProcessorCount, p.regsPerBlock, p.maxThreadsPerBlock,
            p.maxGridSize[0], p.maxGridSize[1], p.maxGridSize[2], p.maxThreadsDim[0],
            p.maxThreadsDim[1], p.maxThreadsDim[2]);
        x += buf;
    }
    x += "</gpus>\n";
    *xml = x;
    return RC_OK;
}

// Demosaicing or fit on the connection's stream: device copies, the kernel,
// the copy back.
rc_status run_device_task(const rc_wire_request& r, const uint8_t* in, uint8_t* out,
                          hipStream_t st) {
    void* d_in = nullptr;
    void* d_out = nullptr;
    rc_status rs = RC_OK;
    hipError_t e = hipMalloc(&d_in, (size_t)r.data_bytes);
    if (e == hipSuccess) e = hipMalloc(&d_out, (size_t)r.result_bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_in, in, (size_t)r.data_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        if (r.task == RC_TASK_BILINEAR_DEMOSAIC) {
            rs = rc_demosaic((const uint16_t*)d_in, (int32_t)r.images, (int32_t)r.height,
                             (int32_t)r.width, (uint16_t*)d_out, st);
        } else if (r.task == RC_TASK_GRADIENT_DEMOSAIC) {
            rs = rc_demosaic_gradient((const uint16_t*)d_in, (int32_t)r.images,
                                      (int32_t)r.height, (int32_t)r.width, (uint16_t*)d_out, st);
        } else {
            const size_t xb = (size_t)(r.bands * r.points * r.detectors) * 8;
            rs = rc_fit((const double*)d_in, (const double*)((const uint8_t*)d_in + xb),
                        (int32_t)r.bands, (int32_t)r.points, (int32_t)r.detectors,
                        (int32_t)r.order, (double*)d_out, st);
        }
        if (rs == RC_OK)
            e = hipMemcpyAsync(out, d_out, (size_t)r.result_bytes, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (d_in) (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    if (e == hipErrorOutOfMemory) return RC_ENOMEM;
    if (e != hipSuccess) return hip_fail(e);
    return rs;
}

void serve_connection(rc_wire* w, rc_wire_conn* conn) {
    const int fd = conn->fd;
    (void)hipSetDevice(w->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    uint8_t h[RC_WIRE_HEADER_BYTES];
    while (!w->stopping.load()) {
        bool eof = false;
        if (!recv_all(fd, h, sizeof h, &eof)) break;
        rc_wire_request r;
        rc_status ps = rc_wire_parse(h, &r);
        // Both buffers are pinned host memory sized by the client's header:
        // bound the answer too (a LUT answer can be far larger than its input).
        if (ps == RC_OK && (r.data_bytes > w->opts.max_data_bytes ||
                            r.result_bytes > w->opts.max_data_bytes))
            ps = RC_ENOMEM;
        if (ps != RC_OK || !st) {
            reply(fd, h, ps != RC_OK ? ps : RC_EHIP, nullptr, 0);
            break;  // the length of the data that may follow is unknown
        }
        uint8_t* in = r.data_bytes ? (uint8_t*)rc_host_alloc((size_t)r.data_bytes) : nullptr;
        uint8_t* out = r.result_bytes ? (uint8_t*)rc_host_alloc((size_t)r.result_bytes) : nullptr;
        if ((r.data_bytes && !in) || (r.result_bytes && !out)) {
            rc_host_free(in);
            rc_host_free(out);
            reply(fd, h, RC_ENOMEM, nullptr, 0);
            break;
        }
        if (r.data_bytes && !recv_all(fd, in, (size_t)r.data_bytes, nullptr)) {
            rc_host_free(in);
            rc_host_free(out);
            break;
        }
        rc_status rs = RC_OK;
        std::string xml;
        const void* result = out;
        uint64_t result_bytes = r.result_bytes;
        if (r.task == RC_TASK_LUT_CORRECTION) {
            rc_host_job j{};
            const size_t rows = (size_t)(r.bands * r.detectors);
            const size_t px = rows * (size_t)r.lines;
            j.coeffs = (const double*)in;
            j.dn = (const uint16_t*)(in + rows * 32);
            j.out = (uint16_t*)out;
            j.lut = r.want_lut ? (uint16_t*)(out + px * 2) : nullptr;
            j.lines = r.lines;
            j.detectors = (int32_t)r.detectors;
            j.bands = (int32_t)r.bands;
            j.levels = (int32_t)r.levels;
            uint64_t id = 0;
            rs = rc_server_submit(w->srv, &j, &id);
            if (rs == RC_OK) rs = rc_server_wait(w->srv, id, nullptr);
        } else if (r.task == RC_TASK_GPU_INFO) {
            rs = gpu_info(&xml);
            result = xml.data();
            result_bytes = xml.size();
        } else {
            rs = run_device_task(r, in, out, st);
        }
        const bool ok = reply(fd, h, rs, result, result_bytes);
        rc_host_free(in);
        rc_host_free(out);
        if (!ok) break;
    }
    if (st) (void)hipStreamDestroy(st);
    {
        std::lock_guard<std::mutex> lk(w->mu);
        ::close(fd);  // under the lock: rc_wire_stop never shuts down a closed descriptor
        conn->fd = -1;
    }
    conn->done.store(true);  // last access to *conn by this thread
}

// Joins and forgets the connections whose threads have finished.
void reap(rc_wire* w) {
    std::list<rc_wire_conn> finished;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        for (auto it = w->conns.begin(); it != w->conns.end();) {
            auto next = std::next(it);
            if (it->done.load()) finished.splice(finished.end(), w->conns, it);
            it = next;
        }
    }
    for (auto& c : finished) c.thread.join();
}

void accept_loop(rc_wire* w) {
    while (!w->stopping.load()) {
        reap(w);
        pollfd pfd{w->fd, POLLIN, 0};
        const int k = ::poll(&pfd, 1, 100);
        if (k <= 0 || !(pfd.revents & POLLIN)) continue;
        const int c = ::accept(w->fd, nullptr, nullptr);
        if (c < 0) continue;
        std::lock_guard<std::mutex> lk(w->mu);
        if (w->stopping.load()) {
            ::close(c);
            break;
        }
        try {
            w->conns.emplace_back();
            rc_wire_conn& conn = w->conns.back();
            conn.fd = c;
            conn.thread = std::thread(serve_connection, w, &conn);
        } catch (...) {
            if (!w->conns.empty() && !w->conns.back().thread.joinable()) w->conns.pop_back();
            ::close(c);
        }
    }
}

}  // namespace
}  // namespace rc

extern "C" {

rc_status rc_wire_start(const rc_wire_opts* o, rc_wire** out) {
    if (!out) return RC_EINVAL;
    *out = nullptr;
    rc_wire_opts opts{};
    if (o) opts = *o;
    if (opts.port < 0 || opts.port > 65535 || opts.any_address < 0 || opts.any_address > 1)
        return RC_EINVAL;
    if (opts.max_data_bytes == 0) opts.max_data_bytes = (uint64_t)8 << 30;
    int dev = 0;
    if (!current_device(&dev)) return RC_EHIP;
    rc_wire* w = new (std::nothrow) rc_wire();
    if (!w) return RC_ENOMEM;
    w->opts = opts;
    w->device = dev;
    rc_server_opts so{};
    so.arena_bytes = opts.arena_bytes;
    rc_status st = rc_server_create(&so, &w->srv);
    if (st != RC_OK) {
        delete w;
        return st;
    }
    w->fd = ::socket(AF_INET, SOCK_STREAM, 0);
    int one = 1;
    sockaddr_in addr{};
    addr.sin_family = AF_INET;
    addr.sin_port = htons((uint16_t)opts.port);
    addr.sin_addr.s_addr = htonl(opts.any_address ? INADDR_ANY : INADDR_LOOPBACK);
    socklen_t len = sizeof addr;
    if (w->fd < 0 || ::setsockopt(w->fd, SOL_SOCKET, SO_REUSEADDR, &one, sizeof one) != 0 ||
        ::bind(w->fd, (sockaddr*)&addr, sizeof addr) != 0 || ::listen(w->fd, 64) != 0 ||
        ::getsockname(w->fd, (sockaddr*)&addr, &len) != 0) {
        if (w->fd >= 0) ::close(w->fd);
        rc_server_destroy(w->srv);
        delete w;
        return RC_EBUSY;
    }
    w->port = ntohs(addr.sin_port);
    try {
        w->acceptor = std::thread(accept_loop, w);
    } catch (...) {
        ::close(w->fd);
        rc_server_destroy(w->srv);
        delete w;
        return RC_ENOMEM;
    }
    *out = w;
    return RC_OK;
}

int32_t rc_wire_port(const rc_wire* w) { return w ? w->port : -1; }

void rc_wire_stop(rc_wire* w) {
    if (!w) return;
    w->stopping.store(true);
    if (w->acceptor.joinable()) w->acceptor.join();
    ::close(w->fd);
    std::list<rc_wire_conn> conns;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        for (auto& c : w->conns)
            if (c.fd >= 0) ::shutdown(c.fd, SHUT_RDWR);  // wake blocked reads
        conns.splice(conns.end(), w->conns);
    }
    for (auto& c : conns) c.thread.join();  // each closes its own descriptor
    rc_server_destroy(w->srv);
    delete w;
}

}  // extern "C"
